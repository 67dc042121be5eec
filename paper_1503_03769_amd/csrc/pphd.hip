// libpphd: C ABI (include/pphd.h) over the HIP kernels in kernels.h.
//
// One filter = one run of the distributed particle PHD filter on one device
// stream.  Every device array lives in the caller's workspace, carved here in a
// fixed order; the library allocates only pinned host staging and events.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pphd.h"
#include "../../include/pphd_mlp.h"
#include "kernels.h"
#include "mlp_internal.h"

using namespace pphd;

namespace {

thread_local std::string g_err;

pphd_status fail(pphd_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
pphd_status fail(pphd_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(PPHD_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

// Tile shape of the two likelihood passes (pphd_set_tuning): particles per
// thread (PT) and measurements per wavefront (the measurement loop is cut into
// at most ZSPLIT_MAX chunks).  Workspace arrays are sized for the smallest PT.
constexpr int PT_DEFAULT_F32 = 8, PT_DEFAULT_F64 = 4, PT_MIN_F32 = 4, PT_MIN_F64 = 2, PR = 1;
constexpr int MZ_DEFAULT = 16;
// workgroups of one bearing-frame pass launch (about what the chip keeps
// resident at these kernels' register use)
constexpr int PASS_WGS_DEFAULT = 1024;

const char* kKernelNames[PPHD_K_COUNT] = {
    "k_predict", "k_cz", "k_cz_combine", "k_weight", "k_finalize", "k_fuse",
    "k_rs_tiles", "k_rs_expand", "k_xchg_gather", "k_xchg_scatter", "k_init", "k_wmax",
    "k_geom", "k_wfinal", "k_birth_weight", "k_mlp_infer", "k_birth_mix", "k_zprep", "k_bk_scatter", "k_bk_back",
};

struct Layout {
    size_t off = 0;
    template <typename P>
    P* take(char* base, size_t bytes)
    {
        off = (off + 255) & ~(size_t)255;
        P* p = base ? reinterpret_cast<P*>(base + off) : nullptr;
        off += bytes;
        return p;
    }
};

}  // namespace

struct pphd_filter {
    pphd_model model;
    DevModel dm;
    int K = 0, cap = 0, max_meas = 0, prec = 0;  // K: groups over all runs
    // runs: a single filter is one run of K groups; a batch holds nruns
    // independent runs whose groups follow each other
    int nruns = 1;
    bool batch = false;
    std::vector<Grp> hgd;         // host copy of the group table
    std::vector<pphd_run_desc> runs;
    std::vector<int> hrun_g0;
    Grp* gd = nullptr;            // device group table [K]
    int* run_g0 = nullptr;        // first group of each run [nruns]
    Grp* rgd = nullptr;           // the record of each run's first group [nruns]
    ZWin* win = nullptr;          // measurement windows of the batched update [nruns]
    int32_t* uwin = nullptr;      // windows as given by the caller [nruns][2]
    uint32_t* dstep = nullptr;    // step counter of captured graphs
    ZPrep zprep{};                // frame-ordered measurements of the bearing-frame passes
    int *zHs = nullptr, *zfls = nullptr;  // H and candidate flags in frame order
    void* zFs = nullptr;                  // F in frame order
    int z_cap = 0;                // measurements the batch's set buffer holds
    int Jmax = 0, M0max = 0;
    int32_t* pin_win = nullptr;
    hipGraph_t graph[2] = {};          // captured batch steps, starting from particle set 0 / 1
    hipGraphExec_t graph_exec[2] = {};
    int graph_next[2] = {0, 1};        // particle set a captured step leaves current
    size_t KC = 0;
    size_t esz = 8;
    hipStream_t stream = nullptr;
    int device = 0;  // the device current at create
    uint64_t seed = 0;
    uint32_t run = 0;
    int phase = 0;  // 0 = created, otherwise a pphd_phase
    int cur = 0;    // which particle set is current
    int last_m = 0;
    uint32_t last_step = 0;
    bool record = false;
    bool births_pending = false;  // birth slots reserved by predict, drawn in update
    // a prediction that waits for the update, whose births' launch carries it
    bool pr_pending = false;
    uint32_t pr_step = 0;
    const uint32_t* pr_dstep = nullptr;
    // learned proposal (birth_proposal 2)
    pphd_mlp* mlp = nullptr;
    bool mix_preset = false;  // pphd_set_birth_mixture outputs wait for the next update
    int mix_preset_m = 0;
    double* mix_tab = nullptr;
    float* mix_raw = nullptr;
    bool timing = false;
    int wt1 = 0, wt2 = 0, wtiles1 = 0, wtiles2 = 0, rtiles = 0, Lmax = 0, tiles256 = 0;
    int pt1 = 0, pt2 = 0, mz = MZ_DEFAULT, wtiles_max = 0;
    int pass_wgs = PASS_WGS_DEFAULT;  // workgroups of a bearing-frame pass launch
    int rs_tiles = 0;                 // 256-slot tiles per resampling workgroup (0: by capacity)
    // device arrays (inside the workspace)
    void* X[2][5] = {};  // component arrays of the two particle sets (X[.][4] with dim 5 only)
    int dim = 4;
    void* W[2] = {};
    int *nsurv = nullptr, *ncur = nullptr, *clampctr = nullptr;
    double* zbuf = nullptr;
    double *p1s = nullptr, *p1w = nullptr;
    int* p1h = nullptr;
    int *zH = nullptr, *zflag = nullptr, *cand = nullptr, *ncand = nullptr;
    void* zF = nullptr;
    double *zC = nullptr, *zdW = nullptr;
    double* zS = nullptr;  // (S, H) of each group's C before the sum over groups (global_cz)
    int* zHg = nullptr;
    double *p2mass = nullptr, *p2max = nullptr, *p2zeta = nullptr;
    double *geo_rho = nullptr, *geo_phi = nullptr, *geo_phib = nullptr, *geo_lw = nullptr;
    int pass_mode = 0;  // PASS_FRAMES / PASS_WRAP / PASS_EXACT, from the model
    void* accp = nullptr;
    double* fmass = nullptr;
    int *fLT = nullptr, *rsS = nullptr, *sel = nullptr;
    double* zeta = nullptr;
    EstimateRec* est = nullptr;
    int* nest = nullptr;
    double *tsum = nullptr, *massq = nullptr;
    double* qtot = nullptr;  // each group's quantised parent total Q in QSLOTS partial sums
    // the expansion of a resampling whose exchange may still be fused into it
    bool rs_pending = false;
    uint32_t rs_step = 0;
    const uint32_t* rs_dstep = nullptr;
    int* counts = nullptr;
    int *bkt = nullptr, *bhist = nullptr, *boff = nullptr;  // bearing-bucket order of the parents
    int* borig = nullptr;  // drawing index of each ordered birth
    bool order_ready = false;  // the last update left the parents' bucket offsets and cleared tile sums
    bool prescattered = false;  // the parents' scatter of the coming resampling ran with the fusion
    bool uneven = false;       // groups of different sizes: the frame passes walk flat item lists
    int *ipre1 = nullptr, *igrp1 = nullptr, *ipre2 = nullptr, *igrp2 = nullptr;  // those lists
    // heavy tiles of the second pass: first-pass kept counts, the groups'
    // item tables and their counts
    int *tkept = nullptr, *witems = nullptr, *wnitems = nullptr;
    void* stage = nullptr;
    // host side
    double* pin_z = nullptr;
    hipEvent_t z_done = nullptr;
    bool z_pending = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;
    double acc_ms[PPHD_K_COUNT] = {};
    long long acc_n[PPHD_K_COUNT] = {};
};

namespace {

// batch: the per-run fields of the model (partitions, births, clutter rate,
// particles per target) are ignored in favour of the run table
bool model_ok(const pphd_model* m, std::string& why, bool batch = false)
{
    if (!m) { why = "model is NULL"; return false; }
    if (m->dim != 4 && m->dim != 5) { why = "dim must be 4 or 5"; return false; }
    if (m->dim == 5 && (!(m->sigma_w >= 0) || !(m->birth_sigma_w >= 0))) { why = "sigma_w, birth_sigma_w must be >= 0"; return false; }
    if (!batch && m->partitions < 1) { why = "partitions must be >= 1"; return false; }
    if (!batch && m->births_per_step < 0) { why = "births_per_step must be >= 0"; return false; }
    if (m->precision != PPHD_FP64 && m->precision != PPHD_FP32) { why = "precision must be 0 or 1"; return false; }
    if (!(m->sigma_r > 0) || !(m->sigma_theta > 0)) { why = "sensor sigmas must be > 0"; return false; }
    if (!(m->p_D >= 0 && m->p_D <= 1) || !(m->p_S >= 0 && m->p_S <= 1)) { why = "p_S, p_D must be in [0,1]"; return false; }
    if (!batch && !(m->clutter_rate >= 0)) { why = "clutter_rate must be >= 0"; return false; }
    if (!(m->r_max > m->r_min) || !(m->th_max > m->th_min)) { why = "empty clutter region"; return false; }
    if (!batch && !(m->particles_per_target > 0)) { why = "particles_per_target must be > 0"; return false; }
    if (!(m->exchange_fraction >= 0 && m->exchange_fraction < 0.5)) { why = "exchange_fraction must be in [0, 0.5)"; return false; }
    if (!(m->birth_mass >= 0) || !(m->init_mass >= 0)) { why = "masses must be >= 0"; return false; }
    if (m->birth_proposal < 0 || m->birth_proposal > 2) { why = "birth_proposal must be 0, 1 or 2"; return false; }
    if (m->birth_proposal != 0 && !(m->birth_alpha >= 0 && m->birth_alpha <= 1)) { why = "birth_alpha must be in [0,1]"; return false; }
    if (m->birth_density != 0 && m->birth_density != 1) { why = "birth_density must be 0 or 1"; return false; }
    if (m->birth_density == 1 && m->birth_proposal != 0) { why = "the Gaussian birth density needs birth_proposal 0"; return false; }
    if (m->birth_density == 1)
        for (int d = 0; d < 4; ++d)
            if (!(m->birth_std[d] > 0)) { why = "birth_std must be > 0"; return false; }
    if (m->global_cz != 0 && m->global_cz != 1) { why = "global_cz must be 0 or 1"; return false; }
    if (m->reserved2 != 0) { why = "reserved fields must be 0"; return false; }
    if (!(m->region[1] > m->region[0]) || !(m->region[3] > m->region[2])) { why = "empty surveillance region"; return false; }
    return true;
}

// Carves every device array from base (or only measures when base == nullptr).
size_t carve(pphd_filter* f, char* base)
{
    Layout L;
    const size_t KC = f->KC, K = f->K, Mx = f->max_meas, es = f->esz;
    for (int b = 0; b < 2; ++b) {
        for (int d = 0; d < f->dim; ++d) f->X[b][d] = L.take<char>(base, KC * es);
        f->W[b] = L.take<char>(base, KC * es);
    }
    f->nsurv = L.take<int>(base, K * 4);
    f->ncur = L.take<int>(base, K * 4);
    f->clampctr = L.take<int>(base, 4);
    f->zbuf = L.take<double>(base, (size_t)f->z_cap * 2 * 8);
    f->gd = L.take<Grp>(base, K * sizeof(Grp));
    f->run_g0 = L.take<int>(base, (size_t)f->nruns * 4);
    f->rgd = L.take<Grp>(base, (size_t)f->nruns * sizeof(Grp));
    f->win = L.take<ZWin>(base, (size_t)f->nruns * sizeof(ZWin));
    f->uwin = L.take<int32_t>(base, (size_t)f->nruns * 8);
    f->dstep = L.take<uint32_t>(base, 4);
    f->zprep.zs = L.take<double>(base, (size_t)f->z_cap * 2 * 8);
    f->zprep.orig = L.take<int>(base, (size_t)f->z_cap * 4);
    f->zprep.pos = L.take<int>(base, (size_t)f->z_cap * 4);
    f->zHs = L.take<int>(base, K * Mx * 4);
    f->zFs = L.take<char>(base, K * Mx * es);
    f->zfls = L.take<int>(base, K * Mx * 4);
    f->zprep.rec = L.take<int>(base, (size_t)f->nruns * 16);
    f->p1s = L.take<double>(base, K * f->wtiles_max * Mx * 8);
    f->p1h = L.take<int>(base, K * f->wtiles_max * Mx * 4);
    f->p1w = L.take<double>(base, K * f->wtiles_max * 8);
    f->zH = L.take<int>(base, K * Mx * 4);
    f->zF = L.take<char>(base, K * Mx * es);
    f->zC = L.take<double>(base, K * Mx * 8);
    f->zdW = L.take<double>(base, K * Mx * 8);
    f->zS = L.take<double>(base, K * Mx * 8);
    f->zHg = L.take<int>(base, K * Mx * 4);
    f->zflag = L.take<int>(base, K * Mx * 4);
    f->cand = L.take<int>(base, K * Mx * 4);
    f->ncand = L.take<int>(base, K * 4);
    f->p2mass = L.take<double>(base, K * f->tiles256 * 8);
    f->p2max = L.take<double>(base, K * f->tiles256 * 8);
    f->geo_rho = L.take<double>(base, KC * 8);
    f->geo_phi = L.take<double>(base, KC * 8);
    f->geo_phib = L.take<double>(base, KC * 8);
    f->geo_lw = L.take<double>(base, KC * 8);
    f->accp = L.take<char>(base, (size_t)ZSPLIT_MAX * KC * es);
    f->p2zeta = L.take<double>(base, K * f->wtiles_max * Mx * 5 * 8);
    f->fmass = L.take<double>(base, K * 8);
    f->fLT = L.take<int>(base, K * 4);
    f->rsS = L.take<int>(base, K * 4);
    f->sel = L.take<int>(base, K * Mx * 4);
    f->zeta = L.take<double>(base, K * Mx * 4 * 8);
    f->est = L.take<EstimateRec>(base, (size_t)f->nruns * Mx * sizeof(EstimateRec));
    f->nest = L.take<int>(base, (size_t)f->nruns * 4);
    f->tsum = L.take<double>(base, K * f->rtiles * 8);
    f->massq = L.take<double>(base, K * 8);
    f->qtot = L.take<double>(base, K * QSLOTS * 8);
    f->counts = L.take<int>(base, KC * 4);
    f->bkt = L.take<int>(base, KC * 4);
    f->borig = L.take<int>(base, KC * 4);
    f->ipre1 = L.take<int>(base, (K + 1) * 4);
    // at most BIRTH_CHUNKS items per tile, each group's span padded to 4
    f->igrp1 = L.take<int>(base, K * (f->wtiles_max * BIRTH_CHUNKS + 3) * 4);
    f->ipre2 = L.take<int>(base, (K + 1) * 4);
    f->igrp2 = L.take<int>(base, K * (f->wtiles_max * BIRTH_CHUNKS + 3) * 4);
    f->tkept = L.take<int>(base, K * f->wtiles_max * 4);
    f->witems = L.take<int>(base, K * f->wtiles_max * BIRTH_CHUNKS * 4);
    f->wnitems = L.take<int>(base, K * 4);
    f->bhist = L.take<int>(base, K * (size_t)f->rtiles * BEARING_BUCKETS * 4);
    f->boff = L.take<int>(base, K * (size_t)f->rtiles * BEARING_BUCKETS * 4);
    f->stage = L.take<char>(base, K * (size_t)f->Lmax * 6 * es);
    if (f->model.birth_proposal == 2) {
        f->mix_tab = L.take<double>(base, (size_t)f->z_cap * 4 * MIX_TAB * 8);
        f->mix_raw = L.take<float>(base, Mx * PPHD_MLP_OUTPUTS * 4);
    }
    return (L.off + 255) & ~(size_t)255;
}

// the single run a plain filter's model describes
pphd_run_desc run_of_model(const pphd_model* m, uint32_t run_id)
{
    pphd_run_desc r;
    std::memset(&r, 0, sizeof r);
    r.partitions = m->partitions;
    r.births_per_step = m->births_per_step;
    r.clutter_rate = m->clutter_rate;
    r.particles_per_target = m->particles_per_target;
    r.run_id = run_id;
    return r;
}

int births_of(const pphd_run_desc& r, int jl)
{
    return r.births_per_step / r.partitions + (jl < r.births_per_step % r.partitions ? 1 : 0);
}

int initial_of(const pphd_run_desc& r)
{
    return std::max(1, (int)std::floor(r.particles_per_target / (double)r.partitions + 0.5));
}

bool runs_ok(const pphd_model* m, const pphd_run_desc* runs, int nruns, std::string& why)
{
    if (!runs || nruns < 1) { why = "a batch needs at least one run"; return false; }
    for (int r = 0; r < nruns; ++r) {
        const pphd_run_desc& d = runs[r];
        if (d.partitions < 1) { why = "run partitions must be >= 1"; return false; }
        if (d.births_per_step < 0) { why = "run births_per_step must be >= 0"; return false; }
        if (!(d.clutter_rate >= 0)) { why = "run clutter_rate must be >= 0"; return false; }
        if (!(d.particles_per_target > 0)) { why = "run particles_per_target must be > 0"; return false; }
        if (d.reserved != 0) { why = "run reserved field must be 0"; return false; }
        // the split masses are divided by one partition count for all runs
        if (m->global_cz && d.partitions != runs[0].partitions) {
            why = "global_cz needs every run to have the same partitions";
            return false;
        }
    }
    return true;
}

void set_geometry(pphd_filter* f, const pphd_model* m, const pphd_run_desc* runs, int nruns, int64_t cap,
                  int32_t max_meas, bool batch)
{
    f->model = *m;
    f->dim = m->dim;
    f->batch = batch;
    f->nruns = nruns;
    f->runs.assign(runs, runs + nruns);
    f->K = 0;
    for (int r = 0; r < nruns; ++r) f->K += runs[r].partitions;
    f->cap = (int)cap;
    f->max_meas = max_meas;
    f->z_cap = batch ? nruns * max_meas : max_meas;
    // group table
    const double area = (m->r_max - m->r_min) * (m->th_max - m->th_min);
    f->hgd.clear();
    f->hrun_g0.clear();
    f->Jmax = 0;
    f->M0max = 0;
    for (int r = 0; r < nruns; ++r) {
        const pphd_run_desc& d = runs[r];
        f->hrun_g0.push_back((int)f->hgd.size());
        for (int jl = 0; jl < d.partitions; ++jl) {
            Grp g;
            std::memset(&g, 0, sizeof g);
            g.jl = jl;
            g.K = d.partitions;
            g.g0 = f->hrun_g0.back();
            g.run = r;
            g.Jj = births_of(d, jl);
            g.M0 = initial_of(d);
            g.rng_run = d.run_id;
            g.kappa = d.clutter_rate / area;
            g.Rj = d.particles_per_target / (double)d.partitions;
            g.gz = m->global_cz ? 1 : 0;
            f->Jmax = std::max(f->Jmax, g.Jj);
            f->M0max = std::max(f->M0max, g.M0);
            f->hgd.push_back(g);
        }
    }
    // groups of clearly different sizes (particles per target or births
    // apart by more than a quarter) walk flat item lists in the frame passes
    double rlo = 1e300, rhi = 0.0;
    int jlo = 1 << 30, jhi = 0;
    for (const Grp& g : f->hgd) {
        rlo = std::min(rlo, g.Rj);
        rhi = std::max(rhi, g.Rj);
        jlo = std::min(jlo, g.Jj);
        jhi = std::max(jhi, g.Jj);
    }
    f->uneven = !f->hgd.empty() && (rhi > 1.25 * rlo || jhi > 1.25 * std::max(jlo, 1) + 1);
    f->prec = m->precision;
    f->esz = m->precision == PPHD_FP64 ? 8 : 4;
    f->KC = (size_t)f->K * (size_t)cap;
    f->pt1 = f->pt2 = f->prec == PPHD_FP64 ? PT_DEFAULT_F64 : PT_DEFAULT_F32;
    const int ptmin = f->prec == PPHD_FP64 ? PT_MIN_F64 : PT_MIN_F32;
    f->wtiles_max = (int)((cap + 64 * ptmin - 1) / (64 * ptmin));
    f->wt1 = 64 * f->pt1;
    f->wt2 = 64 * f->pt2;
    f->wtiles1 = (int)((cap + f->wt1 - 1) / f->wt1);
    f->wtiles2 = (int)((cap + f->wt2 - 1) / f->wt2);
    f->rtiles = (int)((cap + 256 * PR - 1) / (256 * PR));
    f->tiles256 = (int)((cap + 255) / 256);
    f->Lmax = (int)std::floor(m->exchange_fraction * (double)cap) + 1;
}

bool sizes_ok(const pphd_run_desc* runs, int nruns, int64_t cap, int32_t max_meas, std::string& why)
{
    // (tiles of 256 slots index the second grid dimension: at most 65535)
    if (cap < 1 || cap > 65535ll * 256) { why = "cap_per_partition out of range"; return false; }
    // k_cz_combine and k_cz_global keep one double per measurement in LDS
    // next to about 13 KB of their own: at most 6144 measurements stay
    // within a workgroup's 64 KB
    if (max_meas < 1 || max_meas > 6144) { why = "max_meas must be in [1, 6144]"; return false; }
    int64_t groups = 0;
    for (int r = 0; r < nruns; ++r) {
        const pphd_run_desc& d = runs[r];
        groups += d.partitions;
        const int M0 = initial_of(d);
        const int Jmax = births_of(d, 0);
        if (M0 > cap) { why = "cap_per_partition < round(R/K) initial particles"; return false; }
        if (Jmax >= cap) { why = "cap_per_partition must exceed the births per group"; return false; }
        if ((int64_t)M0 + Jmax > cap) { why = "cap_per_partition < round(R/K) + births per group"; return false; }
    }
    if (groups * cap > (1ll << 31) - 1) { why = "groups * cap must fit in 31 bits"; return false; }
    if ((int64_t)nruns * max_meas > (1ll << 28)) { why = "runs * max_meas too large"; return false; }
    return true;
}

void fill_devmodel(pphd_filter* f)
{
    const pphd_model& m = f->model;
    DevModel& d = f->dm;
    std::memset(&d, 0, sizeof d);
    const double two_pi = 2.0 * 3.14159265358979323846;
    d.T = m.T;
    d.sigma_a = m.sigma_a;
    d.sx = m.sensor_x;
    d.sy = m.sensor_y;
    d.pS = m.p_S;
    d.pD = m.p_D;
    d.nu = 1.0 - m.p_D;
    // the smallest clutter density of the runs decides the pass mode
    d.kappa = f->hgd[0].kappa;
    for (const Grp& g : f->hgd) d.kappa = std::min(d.kappa, g.kappa);
    // one C over all groups: the groups split the PHD, each carrying 1/K of
    // the initial and birth masses (every run has the same K)
    const double share = m.global_cz ? (double)f->hgd[0].K : 1.0;
    d.birth_mass = m.global_cz ? m.birth_mass / share : m.birth_mass;
    d.reg0 = m.region[0];
    d.reg1 = m.region[1];
    d.reg2 = m.region[2];
    d.reg3 = m.region[3];
    d.sigma_v = m.birth_sigma_v;
    d.init_mass = m.global_cz ? m.init_mass / share : m.init_mass;
    d.Rj = f->hgd[0].Rj;
    d.xfrac = m.exchange_fraction;
    const double c = std::sqrt(std::log2(std::exp(1.0)) / 2.0);
    d.cr = c / m.sigma_r;
    d.ct = c / m.sigma_theta;
    d.period = two_pi * d.ct;
    d.inv_period = 1.0 / d.period;
    d.wscale = m.p_D / (two_pi * m.sigma_r * m.sigma_theta);
    d.sigma_r = m.sigma_r;
    d.sigma_th = m.sigma_theta;
    d.inv_area = 1.0 / ((m.region[1] - m.region[0]) * (m.region[3] - m.region[2]));
    d.alpha = m.birth_alpha;
    d.proposal = m.birth_proposal;
    d.density = m.birth_density;
    d.dim = m.dim;
    d.sigma_w = m.sigma_w;
    d.birth_sigma_w = m.birth_sigma_w;
    for (int k = 0; k < 4; ++k) {
        d.bmean[k] = m.birth_mean[k];
        d.bstd[k] = m.birth_std[k];
    }
    d.K = f->K;  // groups over all runs
    // per-slot grids (tiles, groups) for groups of clearly different sizes
    // (the second grid dimension holds at most 65535 groups)
    d.tile_major = f->uneven && f->K <= 65535 ? 1 : 0;
    d.J = f->Jmax;
    d.cap = f->cap;
    d.M0 = f->M0max;
    // Bearing frames evaluate each residual without the 2 pi wrap.  A pair
    // whose frame residual needs the wrap has a wrapped residual of at least
    // pi/2, so its term is at most 2^-(pi/2 c_t)^2; the frames are exact only
    // when every such term underflows the storage type: (pi/2 c_t)^2 above
    // 160 in float (underflow at 2^-150; sigma_theta below about 0.1 rad) and
    // above 1100 in double (2^-1075; sigma_theta below about 0.04 rad).
    // Otherwise every pair takes the wrapped residual.
    const double half = 0.5 * 3.14159265358979323846 * d.ct;
    const double wrap_cut = f->prec == PPHD_FP64 ? 1100.0 : 160.0;
    f->pass_mode = d.kappa > 0.0 ? (half * half > wrap_cut ? PASS_FRAMES : PASS_WRAP) : PASS_EXACT;
    d.key0 = (uint32_t)f->seed;
    d.key1 = (uint32_t)(f->seed >> 32);
    d.run = f->run;
    d.one_run = f->nruns == 1 ? 1 : 0;
}

template <typename T>
SoA<T> soa(pphd_filter* f, int b)
{
    SoA<T> s;
    for (int d = 0; d < 5; ++d) s.x[d] = (T*)f->X[b][d];
    s.w = (T*)f->W[b];
    return s;
}

Geo geo_of(pphd_filter* f)
{
    return Geo{ f->geo_rho, f->geo_phi, f->geo_phib, f->geo_lw };
}

// grid of a per-slot kernel over `tiles` tiles of every group (the order the
// device model names)
dim3 slot_grid(const pphd_filter* f, int tiles)
{
    return f->dm.tile_major ? dim3(tiles, f->K) : dim3(f->K, tiles);
}

// 256-slot tiles per workgroup of the resampling's scatter and expansion: two
// where the capacity spans 4096 or more such workgroups (two reads per
// thread in flight, half the dispatch rounds), one for small filters, whose
// workgroups would not fill the chip
// 256-slot tiles per workgroup of the resampling scatter and expansion: as
// set by pphd_set_launch_shape, else two where the capacity spans at least
// 2^20 slots
int rs_halves(const pphd_filter* f)
{
    if (f->rs_tiles == 1 || f->rs_tiles == 2) return f->rs_tiles;
    return (size_t)f->K * f->cap >= ((size_t)1 << 20) ? 2 : 1;
}

// zsplit of a measurement count, as the passes derive it
int host_zsplit(int M, int mz)
{
    const int z = (M + mz - 1) / mz;
    return z < 1 ? 1 : (z > ZSPLIT_MAX ? ZSPLIT_MAX : z);
}

// Measurements of an update: one run's set (win == nullptr, M measurements)
// or a batch's concatenated sets with per-run windows (zrows rows in dz).
// dstep: the device step counter when the launches are captured in a graph.
struct UpdArgs {
    const double* dz;
    int M;
    const ZWin* win;
    int zrows;
    const uint32_t* dstep;
};

hipEvent_t take_event(pphd_filter* f)
{
    if (!f->ev_pool.empty()) {
        hipEvent_t e = f->ev_pool.back();
        f->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch helper: optional start/stop events around the launch, then an error check.
template <typename F>
pphd_status launch(pphd_filter* f, int cls, F&& fn)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (f->timing) {
        a = take_event(f);
        b = take_event(f);
        if (a && b) HIP_TRY(hipEventRecord(a, f->stream));
    }
    fn();
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PPHD_EDEVICE, "%s launch failed: %s", kKernelNames[cls], hipGetErrorString(e));
    if (f->timing && a && b) {
        HIP_TRY(hipEventRecord(b, f->stream));
        f->ev_used.push_back({ cls, { a, b } });
    }
    return PPHD_OK;
}

#define LAUNCH(f, cls, ...)                                          \
    do {                                                             \
        pphd_status s_ = launch(f, cls, [&]() { __VA_ARGS__; });     \
        if (s_ != PPHD_OK) return s_;                                \
    } while (0)

template <typename T>
pphd_status order_births(pphd_filter* f, bool weights_later);
template <typename T>
bool births_in_one_launch(const pphd_filter* f);
template <typename T>
bool predict_rides(const pphd_filter* f);
int predict_parts(const pphd_filter* f);
pphd_status flush_predict(pphd_filter* f);

template <typename T, int PT1, int PT2>
pphd_status run_update(pphd_filter* f, const UpdArgs& a)
{
    const DevModel dm = f->dm;
    SoA<T> st = soa<T>(f, f->cur);
    const Geo geo = geo_of(f);
    const int K = f->K, Mx = f->max_meas;
    const Split s1{ f->wtiles1, f->mz }, s2{ f->wtiles2, f->mz };
    // chunks per tile: exact for one run, the maximum for a batch (waves past
    // a group's own chunk count exit at once)
    const int zs = a.win ? ZSPLIT_MAX : host_zsplit(a.M, f->mz);
    // the measurement preparation of the frame passes rides in the births'
    // one-workgroup-per-group launch when there is one (extra workgroups, one
    // per run), else it has a launch of its own below
    const int zruns = f->pass_mode == PASS_FRAMES ? f->nruns : 0;
    bool zprep_done = false;
    // a pending prediction rides in the births' launch, else it goes first
    if (f->pr_pending && !(f->births_pending && predict_rides<T>(f))) {
        pphd_status ps = flush_predict(f);
        if (ps != PPHD_OK) return ps;
    }
    const int npred = f->pr_pending ? predict_parts(f) : 0;
    f->pr_pending = false;
    if (f->births_pending) {
        // births of the measurement-driven proposals: draw, bearing order
        // (recording each birth's drawing index), weights with the geometry
        const int Jmax = f->Jmax;
        if (Jmax > 0 && (dm.proposal == 1 || dm.proposal == 2)) {
            const int cls = dm.proposal == 1 ? PPHD_K_BIRTH : PPHD_K_BIRTH_MIX;
            if (dm.proposal == 2) {
                // mixture table of this step's measurements: from the outputs
                // the caller set, else from the attached network
                const int rows = a.win ? a.zrows : a.M;
                pphd_status ms = PPHD_OK;
                LAUNCH(f, PPHD_K_MLP_INFER,
                       ms = f->mix_preset ? mlp_head_table(f->model, f->stream, a.dz, f->mix_raw, rows, f->mix_tab)
                                          : mlp_mixture_table(f->mlp, f->stream, a.dz, rows, f->mix_tab));
                if (ms != PPHD_OK) return ms;
            }
            const dim3 gb = slot_grid(f, (Jmax + 255) / 256);
            const double* tab = dm.proposal == 2 ? f->mix_tab : nullptr;
            // FP32 groups of up to BIRTH_FUSED_MAX births of the
            // measurement-driven proposal: drawn, ordered and weighted in one
            // workgroup each; up to 1024 BS: drawn and ordered
            // there, weighted by k_birth_weight; larger ones drawn, put in
            // bucket order, then weighted
            constexpr int BS = sizeof(T) == 4 ? 8 : 4;
            bool weighted = false;
            // (FP64 storage and the mixture proposal, whose density loop wants
            // more wavefronts than a 1024-thread workgroup per group leaves:
            // the weights by their own kernel)
            if constexpr (sizeof(T) == 4) {
                if (Jmax <= BIRTH_FUSED_MAX && dm.proposal == 1) {
                    weighted = true;
                    LAUNCH(f, PPHD_K_BIRTH_ORDER,
                           hipLaunchKernelGGL((k_birth_draw_sort<T, 2, 1, true>), dim3(K + zruns + npred), dim3(1024),
                                              0, f->stream, dm, f->gd, st, geo, f->nsurv, f->ncur, a.dz, tab, a.M,
                                              a.win, f->last_step, a.dstep, f->borig, K, f->zprep, zruns, f->bkt));
                    zprep_done = zruns > 0;
                }
            }
            if (!weighted) {
                if (Jmax <= 1024 * BS) {
                    if (dm.proposal == 1)
                        LAUNCH(f, PPHD_K_BIRTH_ORDER,
                               hipLaunchKernelGGL((k_birth_draw_sort<T, BS, 1, false>), dim3(K + zruns + npred),
                                                  dim3(1024), 0, f->stream, dm, f->gd, st, geo, f->nsurv, f->ncur,
                                                  a.dz, tab, a.M, a.win, f->last_step, a.dstep, f->borig, K,
                                                  f->zprep, zruns, f->bkt));
                    else
                        LAUNCH(f, PPHD_K_BIRTH_ORDER,
                               hipLaunchKernelGGL((k_birth_draw_sort<T, BS, 2, false>), dim3(K + zruns + npred),
                                                  dim3(1024), 0, f->stream, dm, f->gd, st, geo, f->nsurv, f->ncur,
                                                  a.dz, tab, a.M, a.win, f->last_step, a.dstep, f->borig, K,
                                                  f->zprep, zruns, f->bkt));
                    zprep_done = zruns > 0;
                } else {
                    if (dm.proposal == 1)
                        LAUNCH(f, cls,
                               hipLaunchKernelGGL((k_birth_draw<T, 1>), gb, dim3(256), 0, f->stream, dm, f->gd, st,
                                                  f->nsurv, f->ncur, a.dz, tab, a.M, a.win, f->last_step, a.dstep,
                                                  f->bkt));
                    else
                        LAUNCH(f, cls,
                               hipLaunchKernelGGL((k_birth_draw<T, 2>), gb, dim3(256), 0, f->stream, dm, f->gd, st,
                                                  f->nsurv, f->ncur, a.dz, tab, a.M, a.win, f->last_step, a.dstep,
                                                  f->bkt));
                    pphd_status os = order_births<T>(f, true);
                    if (os != PPHD_OK) return os;
                }
                if (dm.proposal == 1)
                    LAUNCH(f, cls,
                           hipLaunchKernelGGL((k_birth_weight<T, 1>), gb, dim3(256), 0, f->stream, dm, f->gd, st, geo,
                                              f->nsurv, f->ncur, f->borig, a.dz, tab, a.M, a.win, f->last_step,
                                              a.dstep));
                else
                    LAUNCH(f, cls,
                           hipLaunchKernelGGL((k_birth_weight<T, 2>), gb, dim3(256), 0, f->stream, dm, f->gd, st, geo,
                                              f->nsurv, f->ncur, f->borig, a.dz, tab, a.M, a.win, f->last_step,
                                              a.dstep));
            }
        }
        f->mix_preset = false;
        f->births_pending = false;
    }
    dim3 g1((f->wtiles1 * zs + 3) / 4, K), g2((f->wtiles2 * zs + 3) / 4, K);
    const ZPrepC zpc{ f->zprep.zs, f->zprep.orig, f->zprep.pos, f->zprep.rec };
    const bool frames = f->pass_mode == PASS_FRAMES;
    const ZSorted<T> zsort{ f->zHs, (T*)f->zFs, f->zfls };
    // frame passes: (K, X) grids whose wavefronts stride over each group's
    // work items, X from the group count (about 4096 wavefronts in all, what
    // the chip holds at these kernels' register use; at most the items a
    // group can have)
    auto xdim = [&](int wtiles) {
        const int64_t most = ((int64_t)wtiles * BIRTH_CHUNKS + 3) / 4, want = (f->pass_wgs + K - 1) / K;
        return (unsigned)std::max<int64_t>(1, std::min(most, want));
    };
    dim3 gl1(K, xdim(f->wtiles1)), gl2(K, xdim(f->wtiles2));
    const int* ipre1 = nullptr;
    const int *igrp1 = nullptr, *ipre2 = nullptr, *igrp2 = nullptr;
    // the second pass splits heavy tiles (item tables from the first pass's
    // kept counts) when both passes use the same tiles and the second pass
    // finalizes the weights itself
    const bool split = frames && PT2 % 4 == 0 && f->wt1 == f->wt2;
    const int imax = f->wtiles_max * BIRTH_CHUNKS;
    auto lists = [&](int WT, int* pre, int* grp, const int* cnt) -> pphd_status {
        LAUNCH(f, PPHD_K_ZPREP,
               hipLaunchKernelGGL(k_items_scan, dim3(1), dim3(1024), 0, f->stream, f->ncur, f->nsurv, K, WT, pre,
                                  cnt));
        LAUNCH(f, PPHD_K_ZPREP, hipLaunchKernelGGL(k_items_fill, dim3(K), dim3(256), 0, f->stream, pre, grp));
        return PPHD_OK;
    };
    if (f->pass_mode == PASS_FRAMES && f->uneven) {
        pphd_status ls = lists(f->wt1, f->ipre1, f->igrp1, nullptr);
        if (ls != PPHD_OK) return ls;
        ipre1 = f->ipre1;
        igrp1 = f->igrp1;
        if (split) {
            // the second pass's lists follow its item tables (after the combine)
            ipre2 = f->ipre2;
            igrp2 = f->igrp2;
        } else if (f->wt2 != f->wt1) {
            ls = lists(f->wt2, f->ipre2, f->igrp2, nullptr);
            if (ls != PPHD_OK) return ls;
            ipre2 = f->ipre2;
            igrp2 = f->igrp2;
        } else {
            ipre2 = ipre1;
            igrp2 = igrp1;
        }
        gl1 = dim3(f->pass_wgs);
        gl2 = dim3(f->pass_wgs);
    }
    if (f->pass_mode == PASS_FRAMES) {
        if (!zprep_done)
            LAUNCH(f, PPHD_K_ZPREP,
                   hipLaunchKernelGGL(k_zprep, dim3(f->nruns), dim3(256), 0, f->stream, dm, a.dz, a.M, a.win,
                                      f->zprep));
        LAUNCH(f, PPHD_K_CZ,
               hipLaunchKernelGGL((k_cz_frames<T, PT1>), gl1, dim3(256), 0, f->stream, dm, f->gd, geo,
                                  (const T*)st.w, f->ncur, a.M, a.win, zpc, Mx, s1, f->p1s, f->p1h, f->p1w,
                                  f->nsurv, K, ipre1, igrp1, (const int*)f->zprep.rec, split ? f->tkept : nullptr));
    } else if (f->pass_mode == PASS_WRAP) {
        LAUNCH(f, PPHD_K_CZ,
               hipLaunchKernelGGL((k_cz<T, PT1, PASS_WRAP>), g1, dim3(256), 0, f->stream, dm, f->gd, geo,
                                  (const T*)st.w, f->ncur, a.dz, a.M, a.win, Mx, s1, f->p1s, f->p1h, f->p1w));
    } else {
        LAUNCH(f, PPHD_K_CZ,
               hipLaunchKernelGGL((k_cz<T, PT1, PASS_EXACT>), g1, dim3(256), 0, f->stream, dm, f->gd, geo,
                                  (const T*)st.w, f->ncur, a.dz, a.M, a.win, Mx, s1, f->p1s, f->p1h, f->p1w));
    }
    const bool global = f->model.global_cz != 0;
    LAUNCH(f, PPHD_K_CZ_COMBINE,
           hipLaunchKernelGGL((k_cz_combine<T>), dim3(K), dim3(1024), (size_t)Mx * sizeof(double), f->stream, dm,
                              f->gd, f->ncur, a.M, a.win, frames ? f->zprep.pos : nullptr, zsort, Mx, f->wtiles1,
                              f->wt1, f->p1s, f->p1h, f->p1w, global ? f->zHg : f->zH,
                              (T*)f->zF, f->zC, f->zdW, f->zflag, f->cand, f->ncand, global ? f->zS : nullptr,
                              f->nsurv, (const int*)f->tkept, split ? f->witems : nullptr, imax, f->wt2, f->wnitems));
    if (split && f->uneven) {
        pphd_status ls = lists(f->wt2, f->ipre2, f->igrp2, f->wnitems);
        if (ls != PPHD_OK) return ls;
    }
    if (global)
        LAUNCH(f, PPHD_K_CZ_COMBINE,
               hipLaunchKernelGGL((k_cz_global<T>), dim3(K), dim3(1024), (size_t)Mx * sizeof(double), f->stream, dm,
                                  f->gd, f->ncur, a.M, a.win, frames ? f->zprep.pos : nullptr, zsort, Mx, f->wtiles1,
                                  f->wt1, (const double*)f->p1w, (const double*)f->zS, (const int*)f->zHg, f->zH,
                                  (T*)f->zF, f->zdW, f->zflag, f->cand, f->ncand));
    // frame passes with wave tiles of whole 256-slot tiles finalize the
    // weights themselves (k_wfinal only for the other passes)
    const bool fused = frames && PT2 % 4 == 0;
    if (f->pass_mode == PASS_FRAMES) {
        const WFin<T> fin{ fused ? 1 : 0, st.w, f->bkt, f->bhist, f->p2mass, f->p2max, f->tiles256 };
        LAUNCH(f, PPHD_K_WEIGHT,
               hipLaunchKernelGGL((k_weight_frames<T, PT2>), gl2, dim3(256), 0, f->stream, dm, f->gd, st, geo,
                                  f->ncur, a.M, a.win, zpc, Mx, s2, f->zHs, (const T*)f->zFs, f->zfls, f->p2zeta,
                                  (T*)f->accp, f->nsurv, K, ipre2, igrp2, fin, (const int*)f->zprep.rec,
                                  split ? (const int*)f->witems : nullptr, imax, (const int*)f->wnitems));
    } else {
        LAUNCH(f, PPHD_K_WEIGHT,
               hipLaunchKernelGGL((k_weight<T, PT2, false>), g2, dim3(256), 0, f->stream, dm, f->gd, st, geo, f->ncur,
                                  a.dz, a.M, a.win, Mx, s2, f->zH, (const T*)f->zF, f->zflag, f->p2zeta,
                                  (T*)f->accp));
    }
    if (!fused)
        LAUNCH(f, PPHD_K_WFINAL,
               hipLaunchKernelGGL((k_wfinal<T>), slot_grid(f, f->tiles256), dim3(256), 0, f->stream, dm, f->gd, st.w,
                                  f->ncur, (const T*)f->accp, a.M, a.win, frames ? (1 << 30) : f->mz, f->tiles256,
                                  f->p2mass, f->p2max, (const T*)st.x[0], (const T*)st.x[2], f->bkt, f->bhist,
                                  frames ? f->wt2 : 0, f->nsurv));
    LAUNCH(f, PPHD_K_FINALIZE,
           hipLaunchKernelGGL(k_finalize<4>, dim3(K), dim3(256), 0, f->stream, f->gd, f->ncur, f->tiles256, f->p2mass,
                              f->p2max, a.M, a.win, Mx, f->wtiles2, f->wt2, f->p2zeta, f->cand, f->ncand, f->fmass,
                              f->fLT, f->rsS, f->sel, f->zeta, f->rtiles, f->bhist, f->boff, f->tsum, f->qtot));
    // k_wfinal and k_finalize have prepared the resampling's parent order
    f->order_ready = true;
    f->prescattered = false;
    return PPHD_OK;
}

// the tile shapes pphd_set_tuning accepts
pphd_status dispatch_update(pphd_filter* f, const UpdArgs& a)
{
#define PPHD_CASE(T, A, B) \
    if (f->pt1 == A && f->pt2 == B) return run_update<T, A, B>(f, a);
    if (f->prec == PPHD_FP64) {
        PPHD_CASE(double, 2, 2) PPHD_CASE(double, 2, 4) PPHD_CASE(double, 2, 8)
        PPHD_CASE(double, 4, 2) PPHD_CASE(double, 4, 4) PPHD_CASE(double, 4, 8)
        PPHD_CASE(double, 8, 2) PPHD_CASE(double, 8, 4) PPHD_CASE(double, 8, 8)
    } else {
        PPHD_CASE(float, 4, 4) PPHD_CASE(float, 4, 8) PPHD_CASE(float, 4, 16)
        PPHD_CASE(float, 8, 4) PPHD_CASE(float, 8, 8) PPHD_CASE(float, 8, 16)
        PPHD_CASE(float, 16, 4) PPHD_CASE(float, 16, 8) PPHD_CASE(float, 16, 16)
    }
#undef PPHD_CASE
    return fail(PPHD_EINVAL, "no kernel for tile shape %d/%d", f->pt1, f->pt2);
}

pphd_status flush_resample(pphd_filter* f);

// births of a measurement-driven proposal drawn and ordered by
// k_birth_draw_sort, one workgroup per group (the update's launch that can
// also carry the survivors' prediction: for filters of up to
// PREDICT_RIDE_SLOTS slots, where saving a launch pays; larger ones predict
// in k_predict's own launch, whose 256-thread workgroups run at the
// occupancy of the prediction's registers rather than the births')
constexpr int64_t PREDICT_RIDE_SLOTS = (int64_t)1 << 23;
template <typename T>
bool births_in_one_launch(const pphd_filter* f)
{
    constexpr int BS = sizeof(T) == 4 ? 8 : 4;
    return (f->dm.proposal == 1 || f->dm.proposal == 2) && f->Jmax > 0 && f->Jmax <= 1024 * BS;
}
template <typename T>
bool predict_rides(const pphd_filter* f)
{
    return births_in_one_launch<T>(f) && (int64_t)f->K * f->cap <= PREDICT_RIDE_SLOTS;
}

// workgroups of 2048 slots that predict every group's survivors
int predict_parts(const pphd_filter* f) { return f->K * ((f->cap + 2047) / 2048); }

template <typename T>
pphd_status launch_predict(pphd_filter* f, uint32_t step, const uint32_t* dstep)
{
    dim3 g = slot_grid(f, (f->cap + 255) / 256);
    LAUNCH(f, PPHD_K_PREDICT,
           hipLaunchKernelGGL((k_predict<T>), g, dim3(256), 0, f->stream, f->dm, f->gd, soa<T>(f, f->cur), geo_of(f),
                              f->nsurv, f->ncur, step, dstep, f->bkt));
    return PPHD_OK;
}

// a prediction still waiting for the update, launched on its own
pphd_status flush_predict(pphd_filter* f)
{
    if (!f->pr_pending) return PPHD_OK;
    f->pr_pending = false;
    return f->prec == PPHD_FP64 ? launch_predict<double>(f, f->pr_step, f->pr_dstep)
                                : launch_predict<float>(f, f->pr_step, f->pr_dstep);
}

template <typename T>
pphd_status run_predict(pphd_filter* f, uint32_t step, const uint32_t* dstep)
{
    pphd_status fs = flush_resample(f);
    if (fs != PPHD_OK) return fs;
    if (predict_rides<T>(f)) {
        // the update draws the births in one launch per step; the survivors'
        // prediction rides in it (it needs nothing the births change)
        f->pr_pending = true;
        f->pr_step = step;
        f->pr_dstep = dstep;
        return PPHD_OK;
    }
    dim3 g = slot_grid(f, (f->cap + 255) / 256);
    LAUNCH(f, PPHD_K_PREDICT,
           hipLaunchKernelGGL((k_predict<T>), g, dim3(256), 0, f->stream, f->dm, f->gd, soa<T>(f, f->cur), geo_of(f),
                              f->nsurv, f->ncur, step, dstep, f->bkt));
    // births of the birth density are drawn by k_predict
    if (f->dm.proposal == 0) return order_births<T>(f, false);
    return PPHD_OK;
}

template <typename T>
pphd_status run_init(pphd_filter* f)
{
    dim3 g = slot_grid(f, (f->M0max + 255) / 256);
    LAUNCH(f, PPHD_K_INIT,
           hipLaunchKernelGGL((k_init<T>), g, dim3(256), 0, f->stream, f->dm, f->gd, soa<T>(f, f->cur), f->nsurv));
    return PPHD_OK;
}

// Stable bearing-bucket order of the slots [first_j, ncur_j) of every group,
// from the current particle set into the other one (first == nullptr: every
// slot).  tiles: 256-slot tiles to cover the longest range.
// parents (first == nullptr): the scatter also forms the resampling's tile
// sums, and the histogram and offsets come from the update when it left them
// fuse (parents, with the update's offsets ready): the launch also runs the
// fusion of Step 4 in its first workgroups
template <typename T>
pphd_status bucket_order(pphd_filter* f, int cls, const int* first, int tiles, int* orig = nullptr,
                         const FuseArgs* fuse = nullptr)
{
    SoA<T> cur = soa<T>(f, f->cur), oth = soa<T>(f, 1 - f->cur);
    const bool parents = first == nullptr;
    FuseArgs fa{};
    int frows = 0;
    if (fuse && parents && f->order_ready) {
        fa = *fuse;
        frows = (fa.nruns + f->K - 1) / f->K;
    }
    dim3 g = slot_grid(f, tiles);
    if (!parents || !f->order_ready) {
        LAUNCH(f, cls,
               hipLaunchKernelGGL((k_bk_hist<T>), g, dim3(256), 0, f->stream, f->dm, cur, first, f->ncur, f->rtiles,
                                  f->bkt, f->bhist, parents ? 0 : 1));
        LAUNCH(f, cls,
               hipLaunchKernelGGL(k_bk_scan, dim3(f->K), dim3(1024), 0, f->stream, first, f->ncur, f->rtiles,
                                  f->bhist, f->boff, parents ? f->tsum : nullptr, f->qtot));
    }
    if (rs_halves(f) == 2)
        LAUNCH(f, cls,
               hipLaunchKernelGGL((k_bk_scatter<T, 2>), slot_grid(f, (tiles + 1) / 2 + frows), dim3(256), 0, f->stream,
                                  f->dm, cur, oth, first, f->ncur, f->rtiles, f->bkt, f->boff, f->rsS,
                                  parents ? f->tsum : nullptr, orig, f->qtot, fa, frows));
    else
        LAUNCH(f, cls,
               hipLaunchKernelGGL((k_bk_scatter<T, 1>), slot_grid(f, tiles + frows), dim3(256), 0, f->stream, f->dm,
                                  cur, oth, first, f->ncur, f->rtiles, f->bkt, f->boff, f->rsS,
                                  parents ? f->tsum : nullptr, orig, f->qtot, fa, frows));
    if (parents) f->order_ready = false;
    return PPHD_OK;
}

// the births of every group (slots [nsurv_j, ncur_j)) in bearing-bucket order
// once drawn (in place, or sorted into the other set and back), with their
// geometry; weights_later: the births' weights (and so their geometry) come
// after the order, which then records each ordered slot's drawing index in
// borig
template <typename T>
pphd_status order_births(pphd_filter* f, bool weights_later)
{
    if (f->Jmax <= 0) return PPHD_OK;
    int* orig = weights_later ? f->borig : nullptr;
    const int geo_now = weights_later ? 0 : 1;
    // up to 1024 BS births per group: one workgroup per group, in place
    constexpr int BS = sizeof(T) == 4 ? 8 : 4;
    if (f->Jmax <= 1024 * BS) {
        LAUNCH(f, PPHD_K_BIRTH_ORDER,
               hipLaunchKernelGGL((k_birth_sort<T, BS>), dim3(f->K), dim3(1024), 0, f->stream, f->dm,
                                  soa<T>(f, f->cur), geo_of(f), f->nsurv, f->ncur, orig, geo_now, f->bkt));
        return PPHD_OK;
    }
    const int bt = (f->Jmax + 255) / 256;
    pphd_status s = bucket_order<T>(f, PPHD_K_BIRTH_ORDER, f->nsurv, bt, orig);
    if (s != PPHD_OK) return s;
    LAUNCH(f, PPHD_K_BIRTH_ORDER,
           hipLaunchKernelGGL((k_bk_back<T>), slot_grid(f, bt), dim3(256), 0, f->stream, f->dm, soa<T>(f, 1 - f->cur),
                              soa<T>(f, f->cur), geo_of(f), f->nsurv, f->ncur, geo_now));
    return PPHD_OK;
}

template <typename T>
pphd_status run_resample(pphd_filter* f, uint32_t step, const uint32_t* dstep)
{
    // parents into bearing-bucket order (into the other set), with the
    // resampling's tile sums and group totals (unless the fusion's launch did
    // it); the systematic expansion back into this set waits for the next
    // call, so that an exchange can ride in it
    if (!f->prescattered) {
        pphd_status s = bucket_order<T>(f, PPHD_K_RS_ORDER, nullptr, f->rtiles);
        if (s != PPHD_OK) return s;
    }
    f->prescattered = false;
    f->cur = 1 - f->cur;
    f->rs_pending = true;
    f->rs_step = step;
    f->rs_dstep = dstep;
    return PPHD_OK;
}

// The pending expansion (xchg: with the ring exchange of step xstep fused).
template <typename T>
pphd_status run_expand(pphd_filter* f, bool xchg, uint32_t xstep, const uint32_t* xdstep)
{
    // k_rs_expand: rs_halves 256-slot tiles per workgroup
    const int nh = rs_halves(f);
    dim3 g = slot_grid(f, (f->rtiles + nh - 1) / nh);
    SoA<T> in = soa<T>(f, f->cur), out = soa<T>(f, 1 - f->cur);
    const int x = xchg ? 1 : 0;
    if (nh == 2)
        LAUNCH(f, PPHD_K_RS_EXPAND,
               hipLaunchKernelGGL((k_rs_expand<T, 2>), g, dim3(256), 0, f->stream, f->dm, f->gd, in, out, f->ncur,
                                  f->nsurv, f->rsS, f->tsum, f->rtiles, f->rs_step, f->rs_dstep, f->massq,
                                  f->clampctr, f->counts, f->record ? 1 : 0, (const double*)f->qtot, x, xstep,
                                  xdstep));
    else
        LAUNCH(f, PPHD_K_RS_EXPAND,
               hipLaunchKernelGGL((k_rs_expand<T, 1>), g, dim3(256), 0, f->stream, f->dm, f->gd, in, out, f->ncur,
                                  f->nsurv, f->rsS, f->tsum, f->rtiles, f->rs_step, f->rs_dstep, f->massq,
                                  f->clampctr, f->counts, f->record ? 1 : 0, (const double*)f->qtot, x, xstep,
                                  xdstep));
    f->cur = 1 - f->cur;
    f->rs_pending = false;
    return PPHD_OK;
}

// completes a resampling whose expansion is still pending (no exchange)
pphd_status flush_resample(pphd_filter* f)
{
    if (!f->rs_pending) return PPHD_OK;
    return f->prec == PPHD_FP64 ? run_expand<double>(f, false, 0, nullptr) : run_expand<float>(f, false, 0, nullptr);
}

template <typename T>
pphd_status run_exchange(pphd_filter* f, uint32_t step, const uint32_t* dstep)
{
    bool any = false;
    int kmax = 1;
    for (const pphd_run_desc& r : f->runs) {
        any = any || r.partitions > 1;
        kmax = std::max(kmax, (int)r.partitions);
    }
    // right after the resampling: the exchange rides in its expansion (runs
    // of up to 1024 groups, whose workgroups each form the run's count)
    if (f->rs_pending) {
        if (any && kmax <= 1024) return run_expand<T>(f, true, step, dstep);
        pphd_status s = run_expand<T>(f, false, 0, nullptr);
        if (s != PPHD_OK) return s;
    }
    if (!any) return PPHD_OK;
    SoA<T> st = soa<T>(f, f->cur);
    // runs of at most 1024 groups: one launch over whole strata
    if (kmax <= 1024) {
        const int spb = 1024 / kmax;
        const int64_t gy = ((int64_t)f->Lmax + spb - 1) / spb;
        if (gy <= 65535) {
            LAUNCH(f, PPHD_K_XCHG_SCATTER,
                   hipLaunchKernelGGL((k_xchg_ring<T>), dim3(f->nruns, (unsigned)gy), dim3(1024), 0, f->stream, f->dm,
                                      f->rgd, st, f->nsurv, f->Lmax, step, dstep));
            return PPHD_OK;
        }
    }
    dim3 g = slot_grid(f, (f->Lmax + 255) / 256);
    LAUNCH(f, PPHD_K_XCHG_GATHER,
           hipLaunchKernelGGL((k_xchg_gather<T>), g, dim3(256), 0, f->stream, f->dm, f->gd, st, f->nsurv,
                              (T*)f->stage, f->Lmax, step, dstep));
    LAUNCH(f, PPHD_K_XCHG_SCATTER,
           hipLaunchKernelGGL((k_xchg_scatter<T>), g, dim3(256), 0, f->stream, f->dm, f->gd, st, f->nsurv,
                              (const T*)f->stage, f->Lmax, step, dstep));
    return PPHD_OK;
}

pphd_status check_handle(pphd_filter* f)
{
    if (!f) return fail(PPHD_EINVAL, "filter handle is NULL");
    return PPHD_OK;
}

#define CHECK_HANDLE(f)                          \
    do {                                         \
        pphd_status s_ = check_handle(f);        \
        if (s_ != PPHD_OK) return s_;            \
    } while (0)

pphd_status run_fuse(pphd_filter* f, EstimateRec* out, int cap, int* nout, int M, const ZWin* win)
{
    const FuseArgs fa{ f->rgd, M, win, f->max_meas, f->sel, f->zeta, out, cap, nout, f->nruns };
    LAUNCH(f, PPHD_K_FUSE, hipLaunchKernelGGL(k_fuse, dim3(f->nruns), dim3(256), 0, f->stream, fa));
    return PPHD_OK;
}

// The fusion for estimates left in device memory: right after an update it
// rides in the launch of the coming resampling's parent scatter (which
// needs the same update's results, writes only the other particle set and
// the resampling's sums, and is kept for pphd_resample); otherwise alone.
// The estimates are complete when the stream reaches the launch either way.
template <typename T>
pphd_status run_fuse_device(pphd_filter* f, EstimateRec* out, int cap, int* nout, int M, const ZWin* win)
{
    if (!f->order_ready || f->prescattered) return run_fuse(f, out, cap, nout, M, win);
    const FuseArgs fa{ f->rgd, M, win, f->max_meas, f->sel, f->zeta, out, cap, nout, f->nruns };
    pphd_status s = bucket_order<T>(f, PPHD_K_RS_ORDER, nullptr, f->rtiles, nullptr, &fa);
    if (s != PPHD_OK) return s;
    f->prescattered = true;
    return PPHD_OK;
}

pphd_status fuse_device(pphd_filter* f, EstimateRec* out, int cap, int* nout, int M, const ZWin* win)
{
    return f->prec == PPHD_FP64 ? run_fuse_device<double>(f, out, cap, nout, M, win)
                                : run_fuse_device<float>(f, out, cap, nout, M, win);
}

}  // namespace

extern "C" {

const char* pphd_last_error(void) { return g_err.c_str(); }

const char* pphd_kernel_name(int32_t c) { return (c >= 0 && c < PPHD_K_COUNT) ? kKernelNames[c] : nullptr; }

}  // extern "C"

namespace {

pphd_status size_impl(const pphd_model* model, const pphd_run_desc* runs, int nruns, int64_t cap, int32_t max_meas,
                      bool batch, size_t* bytes)
{
    std::string why;
    if (!model_ok(model, why, batch) || !runs_ok(model, runs, nruns, why) || !sizes_ok(runs, nruns, cap, max_meas, why))
        return fail(PPHD_EINVAL, "%s", why.c_str());
    if (!bytes) return fail(PPHD_EINVAL, "bytes is NULL");
    pphd_filter tmp;
    set_geometry(&tmp, model, runs, nruns, cap, max_meas, batch);
    *bytes = carve(&tmp, nullptr);
    return PPHD_OK;
}

pphd_status create_impl(const pphd_model* model, const pphd_run_desc* runs, int nruns, int64_t cap,
                        int32_t max_meas, void* workspace, size_t workspace_bytes, uint64_t seed, uint32_t run_id,
                        void* stream, bool batch, pphd_filter** out)
{
    std::string why;
    if (!out) return fail(PPHD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!model_ok(model, why, batch) || !runs_ok(model, runs, nruns, why) || !sizes_ok(runs, nruns, cap, max_meas, why))
        return fail(PPHD_EINVAL, "%s", why.c_str());
    if (!workspace) return fail(PPHD_EINVAL, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(PPHD_EINVAL, "workspace must be 256-byte aligned");
    pphd_filter* f = new (std::nothrow) pphd_filter();
    if (!f) return fail(PPHD_ENOMEM, "host allocation failed");
    set_geometry(f, model, runs, nruns, cap, max_meas, batch);
    const size_t need = carve(f, nullptr);
    if (workspace_bytes < need) {
        delete f;
        return fail(PPHD_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    }
    carve(f, (char*)workspace);
    f->seed = seed;
    f->run = run_id;
    f->stream = (hipStream_t)stream;
    if (hipGetDevice(&f->device) != hipSuccess) f->device = 0;
    fill_devmodel(f);
    hipError_t e = hipHostMalloc((void**)&f->pin_z, (size_t)f->z_cap * 2 * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&f->pin_win, (size_t)f->nruns * 8, hipHostMallocDefault);
    if (e != hipSuccess) {
        if (f->pin_z) (void)hipHostFree(f->pin_z);
        delete f;
        return fail(PPHD_EDEVICE, "hipHostMalloc failed: %s", hipGetErrorString(e));
    }
    e = hipEventCreateWithFlags(&f->z_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMemsetAsync(f->clampctr, 0, 4, f->stream);
    if (e == hipSuccess) e = hipMemsetAsync(f->nsurv, 0, (size_t)f->K * 4, f->stream);
    if (e == hipSuccess) e = hipMemsetAsync(f->ncur, 0, (size_t)f->K * 4, f->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(f->gd, f->hgd.data(), f->hgd.size() * sizeof(Grp), hipMemcpyHostToDevice, f->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(f->run_g0, f->hrun_g0.data(), f->hrun_g0.size() * 4, hipMemcpyHostToDevice, f->stream);
    std::vector<Grp> hrgd;
    for (int g0 : f->hrun_g0) hrgd.push_back(f->hgd[g0]);
    if (e == hipSuccess)
        e = hipMemcpyAsync(f->rgd, hrgd.data(), hrgd.size() * sizeof(Grp), hipMemcpyHostToDevice, f->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
    if (e != hipSuccess) {
        (void)hipHostFree(f->pin_z);
        (void)hipHostFree(f->pin_win);
        delete f;
        return fail(PPHD_EDEVICE, "filter set-up failed: %s", hipGetErrorString(e));
    }
    *out = f;
    return PPHD_OK;
}

}  // namespace

extern "C" {

pphd_status pphd_workspace_size(const pphd_model* model, int64_t cap, int32_t max_meas, size_t* bytes)
{
    if (!model) return fail(PPHD_EINVAL, "model is NULL");
    const pphd_run_desc r = run_of_model(model, 0);
    return size_impl(model, &r, 1, cap, max_meas, false, bytes);
}

pphd_status pphd_create(const pphd_model* model, int64_t cap, int32_t max_meas, void* workspace,
                        size_t workspace_bytes, uint64_t seed, uint32_t run_id, void* stream, pphd_filter** out)
{
    if (!model) return fail(PPHD_EINVAL, "model is NULL");
    const pphd_run_desc r = run_of_model(model, run_id);
    return create_impl(model, &r, 1, cap, max_meas, workspace, workspace_bytes, seed, run_id, stream, false, out);
}

pphd_status pphd_batch_workspace_size(const pphd_model* model, const pphd_run_desc* runs, int32_t nruns,
                                      int64_t cap, int32_t max_meas_per_run, size_t* bytes)
{
    return size_impl(model, runs, nruns, cap, max_meas_per_run, true, bytes);
}

pphd_status pphd_batch_create(const pphd_model* model, const pphd_run_desc* runs, int32_t nruns, int64_t cap,
                              int32_t max_meas_per_run, void* workspace, size_t workspace_bytes, uint64_t seed,
                              void* stream, pphd_filter** out)
{
    return create_impl(model, runs, nruns, cap, max_meas_per_run, workspace, workspace_bytes, seed, 0, stream, true,
                       out);
}

pphd_status pphd_destroy(pphd_filter* f)
{
    if (!f) return PPHD_OK;
    (void)hipStreamSynchronize(f->stream);
    if (f->pin_z) (void)hipHostFree(f->pin_z);
    if (f->pin_win) (void)hipHostFree(f->pin_win);
    for (int i = 0; i < 2; ++i) {
        if (f->graph_exec[i]) (void)hipGraphExecDestroy(f->graph_exec[i]);
        if (f->graph[i]) (void)hipGraphDestroy(f->graph[i]);
    }
    if (f->z_done) (void)hipEventDestroy(f->z_done);
    for (auto& u : f->ev_used) {
        (void)hipEventDestroy(u.second.first);
        (void)hipEventDestroy(u.second.second);
    }
    for (auto e : f->ev_pool) (void)hipEventDestroy(e);
    delete f;
    return PPHD_OK;
}

pphd_status pphd_init(pphd_filter* f)
{
    CHECK_HANDLE(f);
    f->rs_pending = false;  // t = 0 replaces whatever a resampling or a prediction left
    f->pr_pending = false;
    f->prescattered = false;
    f->cur = 0;
    pphd_status s = f->prec == PPHD_FP64 ? run_init<double>(f) : run_init<float>(f);
    if (s != PPHD_OK) return s;
    f->phase = PPHD_PHASE_READY;
    return PPHD_OK;
}

pphd_status pphd_predict(pphd_filter* f, uint32_t step)
{
    CHECK_HANDLE(f);
    if (f->phase != PPHD_PHASE_READY && f->phase != PPHD_PHASE_RESAMPLED)
        return fail(PPHD_ESTATE, "predict needs phase READY or RESAMPLED (have %d)", f->phase);
    pphd_status s = f->prec == PPHD_FP64 ? run_predict<double>(f, step, nullptr) : run_predict<float>(f, step, nullptr);
    if (s != PPHD_OK) return s;
    f->last_step = step;
    f->births_pending = f->model.birth_proposal != 0;
    f->phase = PPHD_PHASE_PREDICTED;
    return PPHD_OK;
}

pphd_status pphd_update(pphd_filter* f, const double* z, int32_t m, int32_t z_on_device)
{
    CHECK_HANDLE(f);
    if (f->batch) return fail(PPHD_EINVAL, "a batch is updated with pphd_batch_update");
    if (f->phase != PPHD_PHASE_PREDICTED) return fail(PPHD_ESTATE, "update needs phase PREDICTED (have %d)", f->phase);
    if (m < 0 || m > f->max_meas) return fail(PPHD_EINVAL, "m = %d outside [0, %d]", m, f->max_meas);
    if (m > 0 && !z) return fail(PPHD_EINVAL, "z is NULL");
    if (f->births_pending && f->model.birth_proposal == 2 && f->dm.J > 0) {
        if (f->mix_preset && f->mix_preset_m != m)
            return fail(PPHD_EINVAL, "set_birth_mixture was given %d measurements, update %d", f->mix_preset_m, m);
        if (!f->mix_preset && !f->mlp)
            return fail(PPHD_ESTATE, "birth_proposal 2 needs pphd_attach_mlp or pphd_set_birth_mixture");
    }
    const double* dz = f->zbuf;
    if (m > 0) {
        if (z_on_device) {
            dz = z;
        } else {
            if (f->z_pending) HIP_TRY(hipEventSynchronize(f->z_done));
            std::memcpy(f->pin_z, z, (size_t)m * 2 * sizeof(double));
            HIP_TRY(hipMemcpyAsync(f->zbuf, f->pin_z, (size_t)m * 2 * sizeof(double), hipMemcpyHostToDevice,
                                   f->stream));
            HIP_TRY(hipEventRecord(f->z_done, f->stream));
            f->z_pending = true;
        }
    }
    pphd_status s = dispatch_update(f, UpdArgs{ dz, m, nullptr, m, nullptr });
    if (s != PPHD_OK) return s;
    f->last_m = m;
    f->phase = PPHD_PHASE_UPDATED;
    return PPHD_OK;
}

pphd_status pphd_extract_device(pphd_filter* f, pphd_estimate* d_out, int32_t cap, int32_t* d_n_out)
{
    CHECK_HANDLE(f);
    if (f->phase != PPHD_PHASE_UPDATED || f->last_m < 0)
        return fail(PPHD_ESTATE, "extract needs phase UPDATED after an update (have %d)", f->phase);
    if (!d_n_out || (cap > 0 && !d_out) || cap < 0) return fail(PPHD_EINVAL, "bad output buffers");
    if (f->batch) return fail(PPHD_EINVAL, "a batch's estimates come from pphd_batch_extract(_device)");
    static_assert(sizeof(pphd_estimate) == sizeof(EstimateRec), "record layout");
    return fuse_device(f, (EstimateRec*)d_out, cap, d_n_out, f->last_m, nullptr);
}

pphd_status pphd_extract(pphd_filter* f, pphd_estimate* out, int32_t cap, int32_t* n_out, double* mass)
{
    CHECK_HANDLE(f);
    if (f->phase != PPHD_PHASE_UPDATED || f->last_m < 0)
        return fail(PPHD_ESTATE, "extract needs phase UPDATED after an update (have %d)", f->phase);
    if (!n_out || (cap > 0 && !out) || cap < 0) return fail(PPHD_EINVAL, "bad output buffers");
    if (f->batch) return fail(PPHD_EINVAL, "a batch's estimates come from pphd_batch_extract(_device)");
    pphd_status s = run_fuse(f, f->est, f->max_meas, f->nest, f->last_m, nullptr);
    if (s != PPHD_OK) return s;
    int n = 0;
    HIP_TRY(hipMemcpyAsync(&n, f->nest, 4, hipMemcpyDeviceToHost, f->stream));
    HIP_TRY(hipStreamSynchronize(f->stream));
    const int k = n < cap ? n : cap;
    if (k > 0) HIP_TRY(hipMemcpy(out, f->est, (size_t)k * sizeof(pphd_estimate), hipMemcpyDeviceToHost));
    if (mass) HIP_TRY(hipMemcpy(mass, f->fmass, (size_t)f->K * 8, hipMemcpyDeviceToHost));
    *n_out = k;
    return PPHD_OK;
}

pphd_status pphd_resample(pphd_filter* f, uint32_t step)
{
    CHECK_HANDLE(f);
    if (f->phase != PPHD_PHASE_UPDATED) return fail(PPHD_ESTATE, "resample needs phase UPDATED (have %d)", f->phase);
    pphd_status s =
        f->prec == PPHD_FP64 ? run_resample<double>(f, step, nullptr) : run_resample<float>(f, step, nullptr);
    if (s != PPHD_OK) return s;
    f->phase = PPHD_PHASE_RESAMPLED;
    return PPHD_OK;
}

pphd_status pphd_exchange(pphd_filter* f, uint32_t step)
{
    CHECK_HANDLE(f);
    if (f->phase != PPHD_PHASE_RESAMPLED) return fail(PPHD_ESTATE, "exchange needs phase RESAMPLED (have %d)", f->phase);
    pphd_status s =
        f->prec == PPHD_FP64 ? run_exchange<double>(f, step, nullptr) : run_exchange<float>(f, step, nullptr);
    if (s != PPHD_OK) return s;
    f->phase = PPHD_PHASE_READY;
    return PPHD_OK;
}

pphd_status pphd_read_state(pphd_filter* f, double* x, double* w, int32_t* count)
{
    CHECK_HANDLE(f);
    {
        // work still pending from the last calls first: a resampling's
        // expansion, a prediction waiting for the update
        pphd_status fs = flush_resample(f);
        if (fs == PPHD_OK) fs = flush_predict(f);
        if (fs != PPHD_OK) return fs;
    }
    if (f->phase == 0) return fail(PPHD_ESTATE, "filter has no state yet (call pphd_init or pphd_write_state)");
    const bool current_is_cur = f->phase == PPHD_PHASE_PREDICTED || f->phase == PPHD_PHASE_UPDATED;
    HIP_TRY(hipStreamSynchronize(f->stream));
    if (count) HIP_TRY(hipMemcpy(count, current_is_cur ? f->ncur : f->nsurv, (size_t)f->K * 4, hipMemcpyDeviceToHost));
    std::vector<char> tmp;
    auto fetch = [&](void* src, double* dst) -> pphd_status {
        if (f->prec == PPHD_FP64) {
            HIP_TRY(hipMemcpy(dst, src, f->KC * 8, hipMemcpyDeviceToHost));
        } else {
            tmp.resize(f->KC * 4);
            HIP_TRY(hipMemcpy(tmp.data(), src, f->KC * 4, hipMemcpyDeviceToHost));
            const float* p = (const float*)tmp.data();
            for (size_t i = 0; i < f->KC; ++i) dst[i] = (double)p[i];
        }
        return PPHD_OK;
    };
    if (x)
        for (int d = 0; d < f->dim; ++d) {
            pphd_status s = fetch(f->X[f->cur][d], x + (size_t)d * f->KC);
            if (s != PPHD_OK) return s;
        }
    if (w) {
        pphd_status s = fetch(f->W[f->cur], w);
        if (s != PPHD_OK) return s;
    }
    return PPHD_OK;
}

pphd_status pphd_write_state(pphd_filter* f, const double* x, const double* w, const int32_t* count, int32_t phase)
{
    CHECK_HANDLE(f);
    {
        // work still pending from the last calls first: a resampling's
        // expansion, a prediction waiting for the update
        pphd_status fs = flush_resample(f);
        if (fs == PPHD_OK) fs = flush_predict(f);
        if (fs != PPHD_OK) return fs;
    }
    if (!x || !w || !count) return fail(PPHD_EINVAL, "x, w and count are required");
    if (phase != PPHD_PHASE_READY && phase != PPHD_PHASE_RESAMPLED && phase != PPHD_PHASE_PREDICTED &&
        phase != PPHD_PHASE_UPDATED)
        return fail(PPHD_EINVAL, "unknown phase %d", phase);
    for (int j = 0; j < f->K; ++j)
        if (count[j] < 0 || count[j] > f->cap) return fail(PPHD_EINVAL, "count[%d] = %d outside [0, cap]", j, count[j]);
    if (phase == PPHD_PHASE_READY || phase == PPHD_PHASE_RESAMPLED) {
        for (int j = 0; j < f->K; ++j)
            if (count[j] + f->hgd[j].Jj > f->cap) return fail(PPHD_EINVAL, "count[%d] leaves no room for births", j);
    }
    HIP_TRY(hipStreamSynchronize(f->stream));
    std::vector<float> tmp;
    auto put = [&](void* dst, const double* src) -> pphd_status {
        if (f->prec == PPHD_FP64) {
            HIP_TRY(hipMemcpy(dst, src, f->KC * 8, hipMemcpyHostToDevice));
        } else {
            tmp.resize(f->KC);
            for (size_t i = 0; i < f->KC; ++i) tmp[i] = (float)src[i];
            HIP_TRY(hipMemcpy(dst, tmp.data(), f->KC * 4, hipMemcpyHostToDevice));
        }
        return PPHD_OK;
    };
    for (int d = 0; d < f->dim; ++d) {
        pphd_status s = put(f->X[f->cur][d], x + (size_t)d * f->KC);
        if (s != PPHD_OK) return s;
    }
    pphd_status s = put(f->W[f->cur], w);
    if (s != PPHD_OK) return s;
    const bool is_cur = phase == PPHD_PHASE_PREDICTED || phase == PPHD_PHASE_UPDATED;
    HIP_TRY(hipMemcpy(is_cur ? f->ncur : f->nsurv, count, (size_t)f->K * 4, hipMemcpyHostToDevice));
    f->births_pending = false;  // a written state is complete
    f->order_ready = false;
    f->prescattered = false;
    if (phase == PPHD_PHASE_PREDICTED) {
        dim3 g = slot_grid(f, (f->cap + 255) / 256);
        if (f->prec == PPHD_FP64) {
            LAUNCH(f, PPHD_K_GEOM,
                   hipLaunchKernelGGL((k_geom<double>), g, dim3(256), 0, f->stream, f->dm, soa<double>(f, f->cur),
                                      geo_of(f), f->ncur));
        } else {
            LAUNCH(f, PPHD_K_GEOM,
                   hipLaunchKernelGGL((k_geom<float>), g, dim3(256), 0, f->stream, f->dm, soa<float>(f, f->cur),
                                      geo_of(f), f->ncur));
        }
    }
    if (phase == PPHD_PHASE_UPDATED) {
        if (f->prec == PPHD_FP64) {
            LAUNCH(f, PPHD_K_WMAX,
                   hipLaunchKernelGGL((k_wmax<double>), dim3(f->K), dim3(256), 0, f->stream, f->dm,
                                      (const double*)f->W[f->cur], f->ncur, f->rsS));
        } else {
            LAUNCH(f, PPHD_K_WMAX,
                   hipLaunchKernelGGL((k_wmax<float>), dim3(f->K), dim3(256), 0, f->stream, f->dm,
                                      (const float*)f->W[f->cur], f->ncur, f->rsS));
        }
        f->last_m = -1;  // no update results to extract from
    }
    HIP_TRY(hipStreamSynchronize(f->stream));
    f->phase = phase;
    return PPHD_OK;
}

pphd_status pphd_read_update(pphd_filter* f, double* C, double* dW, double* mass, int32_t* LT)
{
    CHECK_HANDLE(f);
    if (f->batch) return fail(PPHD_EINVAL, "not available for a batch");
    if (f->phase != PPHD_PHASE_UPDATED || f->last_m < 0)
        return fail(PPHD_ESTATE, "no update results (phase %d)", f->phase);
    HIP_TRY(hipStreamSynchronize(f->stream));
    const int M = f->last_m;
    for (int j = 0; j < f->K && M > 0; ++j) {
        if (C) HIP_TRY(hipMemcpy(C + (size_t)j * M, f->zC + (size_t)j * f->max_meas, (size_t)M * 8, hipMemcpyDeviceToHost));
        if (dW) HIP_TRY(hipMemcpy(dW + (size_t)j * M, f->zdW + (size_t)j * f->max_meas, (size_t)M * 8, hipMemcpyDeviceToHost));
    }
    if (mass) HIP_TRY(hipMemcpy(mass, f->fmass, (size_t)f->K * 8, hipMemcpyDeviceToHost));
    if (LT) HIP_TRY(hipMemcpy(LT, f->fLT, (size_t)f->K * 4, hipMemcpyDeviceToHost));
    return PPHD_OK;
}

pphd_status pphd_read_local(pphd_filter* f, int32_t* sel, double* zeta)
{
    CHECK_HANDLE(f);
    if (f->batch) return fail(PPHD_EINVAL, "not available for a batch");
    if (f->phase != PPHD_PHASE_UPDATED || f->last_m < 0)
        return fail(PPHD_ESTATE, "no update results (phase %d)", f->phase);
    HIP_TRY(hipStreamSynchronize(f->stream));
    const int M = f->last_m;
    for (int j = 0; j < f->K && M > 0; ++j) {
        if (sel) HIP_TRY(hipMemcpy(sel + (size_t)j * M, f->sel + (size_t)j * f->max_meas, (size_t)M * 4, hipMemcpyDeviceToHost));
        if (zeta)
            HIP_TRY(hipMemcpy(zeta + (size_t)j * M * 4, f->zeta + (size_t)j * f->max_meas * 4, (size_t)M * 32,
                              hipMemcpyDeviceToHost));
    }
    return PPHD_OK;
}

pphd_status pphd_set_tuning(pphd_filter* f, int32_t pt_cz, int32_t pt_weight, int32_t meas_per_wave)
{
    CHECK_HANDLE(f);
    const bool f64 = f->prec == PPHD_FP64;
    auto ok = [&](int v) { return f64 ? (v == 2 || v == 4 || v == 8) : (v == 4 || v == 8 || v == 16); };
    if (!ok(pt_cz) || !ok(pt_weight))
        return fail(PPHD_EINVAL, "particles per thread must be %s", f64 ? "2, 4 or 8" : "4, 8 or 16");
    if (meas_per_wave < 1 || meas_per_wave > 4096) return fail(PPHD_EINVAL, "meas_per_wave must be in [1, 4096]");
    f->pt1 = pt_cz;
    f->pt2 = pt_weight;
    f->mz = meas_per_wave;
    f->wt1 = 64 * f->pt1;
    f->wt2 = 64 * f->pt2;
    f->wtiles1 = (int)((f->cap + f->wt1 - 1) / f->wt1);
    f->wtiles2 = (int)((f->cap + f->wt2 - 1) / f->wt2);
    return PPHD_OK;
}
pphd_status pphd_set_launch_shape(pphd_filter* f, int32_t pass_workgroups, int32_t rs_tiles)
{
    CHECK_HANDLE(f);
    if (pass_workgroups != 0 && (pass_workgroups < 64 || pass_workgroups > 65535))
        return fail(PPHD_EINVAL, "pass_workgroups must be 0 or in [64, 65535]");
    if (rs_tiles < 0 || rs_tiles > 2) return fail(PPHD_EINVAL, "rs_tiles must be 0, 1 or 2");
    f->pass_wgs = pass_workgroups ? pass_workgroups : PASS_WGS_DEFAULT;
    f->rs_tiles = rs_tiles;
    return PPHD_OK;
}

pphd_status pphd_set_record_counts(pphd_filter* f, int32_t enable)
{
    CHECK_HANDLE(f);
    {
        // work still pending from the last calls first: a resampling's
        // expansion, a prediction waiting for the update
        pphd_status fs = flush_resample(f);
        if (fs == PPHD_OK) fs = flush_predict(f);
        if (fs != PPHD_OK) return fs;
    }
    f->record = enable != 0;
    return PPHD_OK;
}

pphd_status pphd_read_resample(pphd_filter* f, int32_t* counts, double* mass_q, int64_t* clamped)
{
    CHECK_HANDLE(f);
    {
        // work still pending from the last calls first: a resampling's
        // expansion, a prediction waiting for the update
        pphd_status fs = flush_resample(f);
        if (fs == PPHD_OK) fs = flush_predict(f);
        if (fs != PPHD_OK) return fs;
    }
    if (f->phase != PPHD_PHASE_RESAMPLED && f->phase != PPHD_PHASE_READY)
        return fail(PPHD_ESTATE, "no resample results (phase %d)", f->phase);
    HIP_TRY(hipStreamSynchronize(f->stream));
    if (counts) HIP_TRY(hipMemcpy(counts, f->counts, f->KC * 4, hipMemcpyDeviceToHost));
    if (mass_q) HIP_TRY(hipMemcpy(mass_q, f->massq, (size_t)f->K * 8, hipMemcpyDeviceToHost));
    if (clamped) {
        int c = 0;
        HIP_TRY(hipMemcpy(&c, f->clampctr, 4, hipMemcpyDeviceToHost));
        *clamped = c;
    }
    return PPHD_OK;
}

pphd_status pphd_set_timing(pphd_filter* f, int32_t enable)
{
    CHECK_HANDLE(f);
    HIP_TRY(hipStreamSynchronize(f->stream));
    for (auto& u : f->ev_used) {
        f->ev_pool.push_back(u.second.first);
        f->ev_pool.push_back(u.second.second);
    }
    f->ev_used.clear();
    for (int i = 0; i < PPHD_K_COUNT; ++i) {
        f->acc_ms[i] = 0;
        f->acc_n[i] = 0;
    }
    f->timing = enable != 0;
    return PPHD_OK;
}

pphd_status pphd_read_timing(pphd_filter* f, double* ms, int64_t* launches)
{
    CHECK_HANDLE(f);
    HIP_TRY(hipStreamSynchronize(f->stream));
    for (auto& u : f->ev_used) {
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, u.second.first, u.second.second));
        f->acc_ms[u.first] += t;
        f->acc_n[u.first] += 1;
        f->ev_pool.push_back(u.second.first);
        f->ev_pool.push_back(u.second.second);
    }
    f->ev_used.clear();
    for (int i = 0; i < PPHD_K_COUNT; ++i) {
        if (ms) ms[i] = f->acc_ms[i];
        if (launches) launches[i] = f->acc_n[i];
    }
    return PPHD_OK;
}

}  // extern "C"

namespace {

pphd_status batch_windows(pphd_filter* f, const int32_t* dwin, int z_count)
{
    LAUNCH(f, PPHD_K_FINALIZE,
           hipLaunchKernelGGL(k_batch_windows, dim3((f->nruns + 255) / 256), dim3(256), 0, f->stream, dwin, f->nruns,
                              z_count, f->max_meas, f->win));
    return PPHD_OK;
}

template <typename T>
pphd_status step_all(pphd_filter* f, const double* dz, int z_count, const int32_t* dwin, EstimateRec* out, int cap,
                     int* nout)
{
    // one whole step with every kernel reading the step index from the device counter
    pphd_status s = run_predict<T>(f, 0, f->dstep);
    if (s != PPHD_OK) return s;
    f->births_pending = f->model.birth_proposal != 0;
    s = batch_windows(f, dwin, z_count);
    if (s != PPHD_OK) return s;
    s = dispatch_update(f, UpdArgs{ dz, 0, f->win, z_count, f->dstep });
    if (s != PPHD_OK) return s;
    s = run_fuse_device<T>(f, out, cap, nout, 0, f->win);
    if (s != PPHD_OK) return s;
    s = run_resample<T>(f, 0, f->dstep);
    if (s != PPHD_OK) return s;
    s = run_exchange<T>(f, 0, f->dstep);
    if (s != PPHD_OK) return s;
    LAUNCH(f, PPHD_K_FINALIZE, hipLaunchKernelGGL(k_step_next, dim3(1), dim3(64), 0, f->stream, f->dstep));
    return PPHD_OK;
}

}  // namespace

extern "C" {

pphd_status pphd_batch_update(pphd_filter* f, const double* z, int32_t z_count, const int32_t* windows,
                              int32_t on_device)
{
    CHECK_HANDLE(f);
    if (!f->batch) return fail(PPHD_EINVAL, "not a batch (use pphd_update)");
    if (f->phase != PPHD_PHASE_PREDICTED) return fail(PPHD_ESTATE, "update needs phase PREDICTED (have %d)", f->phase);
    if (z_count < 0 || z_count > f->z_cap) return fail(PPHD_EINVAL, "z_count = %d outside [0, %d]", z_count, f->z_cap);
    if (!windows || (z_count > 0 && !z)) return fail(PPHD_EINVAL, "z and windows are required");
    if (f->births_pending && f->model.birth_proposal == 2 && f->Jmax > 0 && !f->mlp)
        return fail(PPHD_ESTATE, "birth_proposal 2 needs pphd_attach_mlp");
    if (f->z_pending) HIP_TRY(hipEventSynchronize(f->z_done));
    const int32_t* dwin = windows;
    if (!on_device) {
        for (int r = 0; r < f->nruns; ++r) {
            const int32_t off = windows[2 * r], cnt = windows[2 * r + 1];
            if (off < 0 || cnt < 0 || cnt > f->max_meas || (int64_t)off + cnt > z_count)
                return fail(PPHD_EINVAL, "window of run %d (offset %d, count %d) outside the set", r, off, cnt);
        }
        std::memcpy(f->pin_win, windows, (size_t)f->nruns * 8);
        HIP_TRY(hipMemcpyAsync(f->uwin, f->pin_win, (size_t)f->nruns * 8, hipMemcpyHostToDevice, f->stream));
        dwin = f->uwin;
    }
    const double* dz = f->zbuf;
    if (z_count > 0) {
        if (on_device) {
            dz = z;
        } else {
            std::memcpy(f->pin_z, z, (size_t)z_count * 16);
            HIP_TRY(hipMemcpyAsync(f->zbuf, f->pin_z, (size_t)z_count * 16, hipMemcpyHostToDevice, f->stream));
        }
    }
    if (!on_device) {
        HIP_TRY(hipEventRecord(f->z_done, f->stream));
        f->z_pending = true;
    }
    pphd_status s = batch_windows(f, dwin, z_count);
    if (s != PPHD_OK) return s;
    s = dispatch_update(f, UpdArgs{ dz, 0, f->win, z_count, nullptr });
    if (s != PPHD_OK) return s;
    f->last_m = -2;  // per-run counts live in the windows
    f->phase = PPHD_PHASE_UPDATED;
    return PPHD_OK;
}

pphd_status pphd_batch_extract_device(pphd_filter* f, pphd_estimate* d_out, int32_t cap, int32_t* d_n_out)
{
    CHECK_HANDLE(f);
    if (!f->batch) return fail(PPHD_EINVAL, "not a batch (use pphd_extract_device)");
    if (f->phase != PPHD_PHASE_UPDATED || f->last_m != -2)
        return fail(PPHD_ESTATE, "extract needs phase UPDATED after an update (have %d)", f->phase);
    if (!d_n_out || !d_out || cap < 1) return fail(PPHD_EINVAL, "bad output buffers");
    return fuse_device(f, (EstimateRec*)d_out, cap, d_n_out, 0, f->win);
}

pphd_status pphd_batch_extract(pphd_filter* f, pphd_estimate* out, int32_t cap, int32_t* n_out, double* mass)
{
    CHECK_HANDLE(f);
    if (!f->batch) return fail(PPHD_EINVAL, "not a batch (use pphd_extract)");
    if (f->phase != PPHD_PHASE_UPDATED || f->last_m != -2)
        return fail(PPHD_ESTATE, "extract needs phase UPDATED after an update (have %d)", f->phase);
    if (!n_out || !out || cap < 1) return fail(PPHD_EINVAL, "bad output buffers");
    pphd_status s = run_fuse(f, f->est, f->max_meas, f->nest, 0, f->win);
    if (s != PPHD_OK) return s;
    std::vector<int> n(f->nruns);
    HIP_TRY(hipMemcpyAsync(n.data(), f->nest, (size_t)f->nruns * 4, hipMemcpyDeviceToHost, f->stream));
    HIP_TRY(hipStreamSynchronize(f->stream));
    for (int r = 0; r < f->nruns; ++r) {
        const int k = std::min(n[r], std::min(cap, f->max_meas));
        if (k > 0)
            HIP_TRY(hipMemcpy(out + (size_t)r * cap, f->est + (size_t)r * f->max_meas, (size_t)k * sizeof(pphd_estimate),
                              hipMemcpyDeviceToHost));
        n_out[r] = k;
    }
    if (mass) HIP_TRY(hipMemcpy(mass, f->fmass, (size_t)f->K * 8, hipMemcpyDeviceToHost));
    return PPHD_OK;
}

pphd_status pphd_batch_capture(pphd_filter* f, const double* d_z, int32_t z_count, const int32_t* d_windows,
                               pphd_estimate* d_out, int32_t cap, int32_t* d_n_out, uint32_t first_step)
{
    CHECK_HANDLE(f);
    if (!f->batch) return fail(PPHD_EINVAL, "not a batch");
    if (f->phase != PPHD_PHASE_READY && f->phase != PPHD_PHASE_RESAMPLED)
        return fail(PPHD_ESTATE, "capture needs phase READY or RESAMPLED (have %d)", f->phase);
    if (f->timing) return fail(PPHD_ESTATE, "disable timing before capturing");
    if (z_count < 0 || z_count > f->z_cap) return fail(PPHD_EINVAL, "z_count = %d outside [0, %d]", z_count, f->z_cap);
    if (!d_windows || !d_out || !d_n_out || cap < 1 || (z_count > 0 && !d_z))
        return fail(PPHD_EINVAL, "bad buffers");
    if (f->model.birth_proposal == 2 && f->Jmax > 0 && !f->mlp)
        return fail(PPHD_ESTATE, "birth_proposal 2 needs pphd_attach_mlp");
    {
        pphd_status fs = flush_resample(f);
        if (fs != PPHD_OK) return fs;
    }
    if (f->z_pending) HIP_TRY(hipEventSynchronize(f->z_done));
    HIP_TRY(hipStreamSynchronize(f->stream));
    HIP_TRY(hipMemcpy(f->dstep, &first_step, 4, hipMemcpyHostToDevice));
    for (int i = 0; i < 2; ++i) {
        if (f->graph_exec[i]) (void)hipGraphExecDestroy(f->graph_exec[i]);
        if (f->graph[i]) (void)hipGraphDestroy(f->graph[i]);
        f->graph_exec[i] = nullptr;
        f->graph[i] = nullptr;
    }
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipStream_t user = f->stream;
    const int cur0 = f->cur;
    pphd_status s = PPHD_OK;
    for (int i = 0; i < 2 && s == PPHD_OK; ++i) {
        f->cur = i;
        f->stream = cs;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            s = fail(PPHD_EDEVICE, "hipStreamBeginCapture failed: %s", hipGetErrorString(e));
            break;
        }
        s = f->prec == PPHD_FP64 ? step_all<double>(f, d_z, z_count, d_windows, (EstimateRec*)d_out, cap, d_n_out)
                                 : step_all<float>(f, d_z, z_count, d_windows, (EstimateRec*)d_out, cap, d_n_out);
        f->graph_next[i] = f->cur;
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        if (s == PPHD_OK && e != hipSuccess) s = fail(PPHD_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
        if (s == PPHD_OK) {
            f->graph[i] = g;
            e = hipGraphInstantiate(&f->graph_exec[i], g, nullptr, nullptr, 0);
            if (e != hipSuccess) s = fail(PPHD_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
    }
    f->stream = user;
    f->cur = cur0;
    f->births_pending = false;
    (void)hipStreamDestroy(cs);
    return s;
}

pphd_status pphd_batch_launch(pphd_filter* f)
{
    CHECK_HANDLE(f);
    {
        // work still pending from the last calls first: a resampling's
        // expansion, a prediction waiting for the update
        pphd_status fs = flush_resample(f);
        if (fs == PPHD_OK) fs = flush_predict(f);
        if (fs != PPHD_OK) return fs;
    }
    if (!f->batch || !f->graph_exec[0] || !f->graph_exec[1]) return fail(PPHD_ESTATE, "no captured step (pphd_batch_capture)");
    if (f->phase != PPHD_PHASE_READY && f->phase != PPHD_PHASE_RESAMPLED)
        return fail(PPHD_ESTATE, "launch needs phase READY or RESAMPLED (have %d)", f->phase);
    HIP_TRY(hipGraphLaunch(f->graph_exec[f->cur], f->stream));
    f->cur = f->graph_next[f->cur];
    f->phase = PPHD_PHASE_READY;
    return PPHD_OK;
}

}  // extern "C"

namespace pphd {
pphd_status set_error(pphd_status s, const char* msg)
{
    g_err = msg;
    return s;
}
}  // namespace pphd

extern "C" {

pphd_status pphd_attach_mlp(pphd_filter* f, pphd_mlp* h)
{
    CHECK_HANDLE(f);
    if (h && f->model.birth_proposal != 2) return fail(PPHD_EINVAL, "the filter's birth_proposal is not 2");
    f->mlp = h;
    return PPHD_OK;
}

pphd_status pphd_set_birth_mixture(pphd_filter* f, const float* raw, int32_t m, int32_t on_device)
{
    CHECK_HANDLE(f);
    if (f->model.birth_proposal != 2 || f->batch) return fail(PPHD_EINVAL, "the filter's birth_proposal is not 2");
    if (f->phase != PPHD_PHASE_PREDICTED) return fail(PPHD_ESTATE, "set_birth_mixture needs phase PREDICTED (have %d)", f->phase);
    if (m < 0 || m > f->max_meas) return fail(PPHD_EINVAL, "m = %d outside [0, %d]", m, f->max_meas);
    if (m > 0 && !raw) return fail(PPHD_EINVAL, "raw is NULL");
    if (m > 0) {
        HIP_TRY(hipMemcpyAsync(f->mix_raw, raw, (size_t)m * PPHD_MLP_OUTPUTS * 4,
                               on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, f->stream));
        if (!on_device) HIP_TRY(hipStreamSynchronize(f->stream));
    }
    f->mix_preset = true;
    f->mix_preset_m = m;
    return PPHD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free update.  pphd_update_noalloc is pphd_update with the first
// likelihood pass's partial sums (per group, wave tile and measurement: the
// scaled sum, its exponent, and per tile the weight sum) in the static device
// array `scratch` instead of the caller's workspace.  Every device holds its
// own copy of the array for the life of the process, and every call on a
// device shares it; nothing in it needs clearing, since the first pass
// writes every partial that the combine reads in the same update.
// ---------------------------------------------------------------------------
constexpr size_t PPHD_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) char scratch[PPHD_SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_DEVICES = 64;
std::mutex scratch_mu;
char* scratch_ptr[SCRATCH_DEVICES] = {};

// The device address of `scratch` on device dev, looked up once per device
// with that device current (host code never passes the array's own name).
pphd_status scratch_on(int dev, char** out)
{
    if (dev < 0 || dev >= SCRATCH_DEVICES) return fail(PPHD_EDEVICE, "device %d has no static scratch slot", dev);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        int cur = 0;
        HIP_TRY(hipGetDevice(&cur));
        if (cur != dev) HIP_TRY(hipSetDevice(dev));
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr)
            return fail(PPHD_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        scratch_ptr[dev] = static_cast<char*>(ptr);
    }
    *out = scratch_ptr[dev];
    return PPHD_OK;
}

}  // namespace

extern "C" {

pphd_status pphd_update_noalloc(pphd_filter* f, const double* z, int32_t m, int32_t z_on_device)
{
    CHECK_HANDLE(f);
    if (f->batch) return fail(PPHD_EINVAL, "a batch is updated with pphd_batch_update");
    if (f->timing) return fail(PPHD_EINVAL, "pphd_update_noalloc records no kernel times (turn timing off)");
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t n = (size_t)f->K * (size_t)f->wtiles_max;
    const size_t bs = up(n * (size_t)f->max_meas * 8), bh = up(n * (size_t)f->max_meas * 4), bw = up(n * 8);
    if (bs + bh + bw > PPHD_SCRATCH_BYTES)
        return fail(PPHD_EINVAL, "the first pass's partials need %zu bytes; the static scratch holds %zu",
                    bs + bh + bw, PPHD_SCRATCH_BYTES);
    char* base = nullptr;
    pphd_status st = scratch_on(f->device, &base);
    if (st != PPHD_OK) return st;
    double* const ks = f->p1s;
    int* const kh = f->p1h;
    double* const kw = f->p1w;
    f->p1s = reinterpret_cast<double*>(base);
    f->p1h = reinterpret_cast<int*>(base + bs);
    f->p1w = reinterpret_cast<double*>(base + bs + bh);
    st = pphd_update(f, z, m, z_on_device);
    f->p1s = ks;
    f->p1h = kh;
    f->p1w = kw;
    return st;
}

}  // extern "C"
