// C ABI of the library (declared in include/nbody.h): argument checks,
// workspace layout, and the host sequence of kernels of each call.  All
// arithmetic runs in the kernels of force.hip and integrate.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>

#include "nbody_internal.h"

using namespace nb;

struct nbody_ctx {
    Ctx c;
};

// Scratch of nbody_force_noalloc: the source records, the one-cluster work
// tables and the split-source partials of one evaluation, in a fixed device
// array instead of a caller workspace.  Each device the library runs on
// holds its own copy until the process ends.  Host code never uses the
// array's name as an address: the device address is looked up once per
// device (scratch_address below) and only that address is passed on.
constexpr int64_t NOALLOC_SCRATCH_BYTES = int64_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int64_t ALIGN = 256;

int64_t align_up(int64_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

bool is_pow2(double x)
{
    if (!(x > 0.0) || !std::isfinite(x))
        return false;
    int e;
    return std::frexp(x, &e) == 0.5;
}

bool config_ok(const nbody_config *cfg, int64_t n)
{
    if (!cfg)
        return false;
    if (!(cfg->eta > 0.0) || !std::isfinite(cfg->eta))
        return false;
    if (!(cfg->eta_init > 0.0) || !std::isfinite(cfg->eta_init))
        return false;
    if (!is_pow2(cfg->dt_min) || !is_pow2(cfg->dt_max) || cfg->dt_min > cfg->dt_max)
        return false;
    if (cfg->precision != NBODY_PREC_MIXED && cfg->precision != NBODY_PREC_FP64 &&
        cfg->precision != NBODY_PREC_FP32PAIR)
        return false;
    if (cfg->n_clusters > 1) {
        const int64_t *o = cfg->cluster_offsets;
        if (!o || o[0] != 0 || o[cfg->n_clusters] != n)
            return false;
        for (int32_t c = 0; c < cfg->n_clusters; ++c)
            if (o[c + 1] <= o[c])
                return false;
    }
    return true;
}

int32_t n_clusters(const nbody_config *cfg) { return cfg->n_clusters > 1 ? cfg->n_clusters : 1; }

int64_t count_chunks(const std::vector<int64_t> &off)
{
    int64_t k = 0;
    for (size_t c = 0; c + 1 < off.size(); ++c)
        k += (off[c + 1] - off[c] + SCHED_CHUNK - 1) / SCHED_CHUNK;
    return k;
}

int fail(Ctx &c, int code, const char *what)
{
    c.last_error = what;
    return code;
}

int hip_fail(Ctx &c, hipError_t e, const char *where)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
    c.last_error = buf;
    return NBODY_EDEVICE;
}

#define HIPCHK(ctx, call)                                  \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess)                              \
            return hip_fail((ctx), e_, #call);             \
    } while (0)

// read the device error word; clear it; map it to a return code
int take_err(Ctx &c)
{
    HIPCHK(c, hipMemcpyAsync(c.h_err, c.d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(c, hipStreamSynchronize(c.stream));
    const uint32_t e = *c.h_err;
    if (!e)
        return NBODY_OK;
    HIPCHK(c, hipMemsetAsync(c.d_err, 0, sizeof(uint32_t), c.stream));
    HIPCHK(c, hipStreamSynchronize(c.stream));
    if (e & ERR_NONFINITE)
        return fail(c, NBODY_ENONFINITE, "non-finite value in the state");
    if (e & ERR_DTMIN)
        return fail(c, NBODY_EDTMIN, "a particle needs a step below dt_min");
    if (e & ERR_LOOP)
        return fail(c, NBODY_EDEVICE, "a grid barrier of the device-resident loop timed out");
    if (e & ERR_STATE)
        return fail(c, NBODY_ESTATE, "the particles of a cluster are not at one time");
    if (e & ERR_LEVELS)
        return fail(c, NBODY_EDEVICE, "the schedule from level counts and the active list disagree");
    return fail(c, NBODY_EINVAL, "index list out of range / not ascending, or a particle is past the target time");
}

// device address of the current device's copy of the scratch array (looked
// up with hipGetSymbolAddress on the first call on each device)
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_addr[NOALLOC_MAX_DEVICES] = {};

hipError_t scratch_address(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        g_scratch_addr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

// Scratch layout of nbody_force_noalloc for n sources: the records of the
// context's precision, seg[2] and off[2]; the split partials follow at the
// returned offset.  With base == nullptr only the size is computed.
int64_t noalloc_layout(int64_t n, int32_t prec, Ctx *c, unsigned char *base, int64_t **seg,
                       int64_t **off)
{
    int64_t o = 0;
    auto take = [&](int64_t bytes) -> unsigned char * {
        unsigned char *p = base ? base + o : nullptr;
        o += align_up(bytes);
        return p;
    };
    const int64_t d = sizeof(double), f = sizeof(float);
    if (prec == NBODY_PREC_MIXED) {
        double **dl[7] = {&c->jm.x, &c->jm.y, &c->jm.z, &c->jm.m, &c->jm.vx, &c->jm.vy, &c->jm.vz};
        for (auto p : dl)
            *p = (double *)take(n * d);
        float **fl[3] = {&c->jm.ax, &c->jm.ay, &c->jm.az};
        for (auto p : fl)
            *p = (float *)take(n * f);
    } else if (prec == NBODY_PREC_FP32PAIR) {
        double **dl[4] = {&c->jp.x, &c->jp.y, &c->jp.z, &c->jp.m};
        for (auto p : dl)
            *p = (double *)take(n * d);
        float **fl[6] = {&c->jp.vx, &c->jp.vy, &c->jp.vz, &c->jp.ax, &c->jp.ay, &c->jp.az};
        for (auto p : fl)
            *p = (float *)take(n * f);
    } else {
        double **dl[10] = {&c->jd.x, &c->jd.y, &c->jd.z, &c->jd.vx, &c->jd.vy,
                           &c->jd.vz, &c->jd.ax, &c->jd.ay, &c->jd.az, &c->jd.m};
        for (auto p : dl)
            *p = (double *)take(n * d);
    }
    *seg = (int64_t *)take(2 * 8);
    *off = (int64_t *)take(2 * 8);
    return o;
}

}  // namespace

// Workspace layout: every array 256-byte aligned.  With base == nullptr
// only the size is computed.
int64_t nb::ws_layout(int64_t n, int32_t nc, int32_t prec, Ctx *c, char *base)
{
    int64_t o = 0;
    auto take = [&](int64_t bytes) -> char * {
        char *p = base ? base + o : nullptr;
        o += align_up(bytes);
        return p;
    };
    const int64_t d = sizeof(double), f = sizeof(float);
    const int64_t part_cap = std::max<int64_t>(2 * n, int64_t(1) << 20);
    const int64_t n_chunks_max = n / SCHED_CHUNK + nc + 1;
    State st{};
    st.pos = (double *)take(3 * n * d);
    st.vel = (double *)take(3 * n * d);
    st.acc = (double *)take(3 * n * d);
    st.jrk = (double *)take(3 * n * d);
    st.snp = (double *)take(3 * n * d);
    st.crk = (double *)take(3 * n * d);
    st.t = (double *)take(n * d);
    st.dt = (double *)take(n * d);
    st.mass = (double *)take(n * d);
    JRecMixed jm{};
    JRecPair32 jp{};
    JRecF64 jd{};
    if (prec == NBODY_PREC_MIXED) {
        double **dl[7] = {&jm.x, &jm.y, &jm.z, &jm.m, &jm.vx, &jm.vy, &jm.vz};
        for (auto p : dl)
            *p = (double *)take(n * d);
        float **fl[3] = {&jm.ax, &jm.ay, &jm.az};
        for (auto p : fl)
            *p = (float *)take(n * f);
    } else if (prec == NBODY_PREC_FP32PAIR) {
        jp.x = (double *)take(n * d);
        jp.y = (double *)take(n * d);
        jp.z = (double *)take(n * d);
        jp.m = (double *)take(n * d);
        float **fl[6] = {&jp.vx, &jp.vy, &jp.vz, &jp.ax, &jp.ay, &jp.az};
        for (auto p : fl)
            *p = (float *)take(n * f);
    } else {
        double **dl[10] = {&jd.x, &jd.y, &jd.z, &jd.vx, &jd.vy, &jd.vz, &jd.ax, &jd.ay, &jd.az, &jd.m};
        for (auto p : dl)
            *p = (double *)take(n * d);
    }
    double *part = (double *)take(10 * part_cap * d);
    int32_t *act = (int32_t *)take(n * 4);
    double *fnew = (double *)take(10 * n * d);
    int64_t *d_off = (int64_t *)take((nc + 1) * 8);
    int32_t *cl_of = nc > 1 ? (int32_t *)take(n * 4) : nullptr;
    int32_t *ch_cl = (int32_t *)take(n_chunks_max * 4);
    int64_t *ch_b = (int64_t *)take((n_chunks_max + 1) * 8);
    uint64_t *tmin = (uint64_t *)take(nc * 8);
    double *tblock = (double *)take(nc * d);
    int32_t *ch_cnt = (int32_t *)take(n_chunks_max * 4);
    uint64_t *ch_min = (uint64_t *)take(n_chunks_max * 8);
    int64_t *ch_pos = (int64_t *)take(n_chunks_max * 8);
    int64_t *seg = (int64_t *)take((nc + 1) * 8);
    int32_t *blk_cl = (int32_t *)take((n + nc + 1) * 4);
    int64_t *blk_first = (int64_t *)take((nc + 1) * 8);
    int64_t *info = (int64_t *)take(64 * 8);
    int64_t *lvl = (int64_t *)take(LVL_WORDS * 8);
    uint64_t *loop_min = (uint64_t *)take(2 * LOOP_GMAX * 8);
    int32_t *loop_cnt = (int32_t *)take(2 * LOOP_GMAX * 4);
    // ensemble plan: grp_of, first, size [LOOP_GMAX each], cl_off [LOOP_GMAX + 1],
    // cl [nc]; part_off, part_cap [LOOP_GMAX each], seg [2 LOOP_GMAX]; results
    int32_t *ens_i32 = nc > 1 ? (int32_t *)take((4 * LOOP_GMAX + 1 + nc) * 4) : nullptr;
    int64_t *ens_i64 = nc > 1 ? (int64_t *)take(4 * LOOP_GMAX * 8) : nullptr;
    unsigned long long *ens_res = nc > 1 ? (unsigned long long *)take(4 * 8) : nullptr;
    uint32_t *loop_bar = (uint32_t *)take(2 * LOOP_BAR_WORDS * 4);
    uint32_t *err = (uint32_t *)take(4);
    const int64_t red_cap = 5 * (n / 256 + 2) + 16;
    double *red = (double *)take(red_cap * d);
    double *phi = (double *)take(n * d);
    if (c) {
        c->st = st;
        c->jm = jm;
        c->jp = jp;
        c->jd = jd;
        c->part = part;
        c->part_cap = part_cap;
        c->act = act;
        c->fnew = fnew;
        c->d_off = d_off;
        c->d_cluster_of = cl_of;
        c->d_chunk_cluster = ch_cl;
        c->d_chunk_begin = ch_b;
        c->d_tmin = tmin;
        c->d_tblock = tblock;
        c->d_chunk_cnt = ch_cnt;
        c->d_chunk_min = ch_min;
        c->d_chunk_pos = ch_pos;
        c->d_seg = seg;
        c->d_blk_cluster = blk_cl;
        c->d_blk_first = blk_first;
        c->d_info = info;
        c->d_lvl = lvl;
        c->d_loop_min = loop_min;
        c->d_loop_cnt = loop_cnt;
        c->d_ens_i32 = ens_i32;
        c->d_ens_i64 = ens_i64;
        c->d_ens_res = ens_res;
        c->d_loop_bar = loop_bar;
        c->d_err = err;
        c->d_red = red;
        c->red_cap = red_cap;
        c->d_phi = phi;
    }
    return o;
}

int nb::prof_begin(Ctx &c, int phase, int64_t n_act, double pairs)
{
    if (!c.prof)
        return -1;
    if (c.prof_pending.size() >= 4096 && prof_collect(c) != hipSuccess)
        return -1;   // bounded event use on long runs
    ProfRec r{};
    r.phase = phase;
    r.n_act = n_act;
    r.pairs = pairs;
    for (hipEvent_t *e : {&r.a, &r.b}) {
        if (!c.prof_pool.empty()) {
            *e = c.prof_pool.back();
            c.prof_pool.pop_back();
        } else if (hipEventCreate(e) != hipSuccess) {
            return -1;
        }
    }
    if (hipEventRecord(r.a, c.stream) != hipSuccess)
        return -1;
    c.prof_pending.push_back(r);
    return (int)c.prof_pending.size() - 1;
}

void nb::prof_end(Ctx &c, int rec)
{
    if (rec < 0 || rec >= (int)c.prof_pending.size())
        return;
    (void)hipEventRecord(c.prof_pending[rec].b, c.stream);
}

hipError_t nb::prof_collect(Ctx &c)
{
    if (c.prof_pending.empty())
        return hipSuccess;
    hipError_t e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess)
        return e;
    for (ProfRec &r : c.prof_pending) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess)
            return e;
        c.prof_ms[r.phase] += ms;
        c.prof_cnt[r.phase] += 1;
        if (r.phase == PH_FORCE) {
            c.prof_pairs += r.pairs;
            c.flog_nact.push_back(r.n_act);
            c.flog_pairs.push_back(r.pairs);
            c.flog_ms.push_back(ms);
        }
        c.prof_pool.push_back(r.a);
        c.prof_pool.push_back(r.b);
    }
    c.prof_pending.clear();
    return hipSuccess;
}

namespace {

// the autotuner has a shape for this active-set size
bool has_tuned(const Ctx &c, int64_t n_act)
{
    if (n_act < 1 || c.tuned.empty())
        return false;
    int b = 0;
    while ((int64_t(1) << (b + 1)) <= n_act)
        ++b;
    return b < (int)c.tuned.size() && c.tuned[b].lpi > 0;
}

int64_t max_cluster(const Ctx &c)
{
    int64_t m = 0;
    for (size_t k = 0; k + 1 < c.off.size(); ++k)
        m = std::max(m, c.off[k + 1] - c.off[k]);
    return m;
}

// force of the active slots described by c.d_seg (and idx) into out
int run_force(Ctx &c, const int32_t *idx, int64_t n_act, int64_t n_act_typ, const ForceOut &out,
              double pairs_hint = -1.0, int64_t n_src = -1, bool reduce = true,
              Launch *used = nullptr, ForceWork *work = nullptr)
{
    Launch L = pick_launch(c, n_act_typ, n_src > 0 ? n_src : max_cluster(c));
    while ((int64_t)L.split * n_act > c.part_cap && L.split > 1)
        L.split >>= 1;
    // a batched launch gets its parallelism from its many clusters: the rule's
    // shape for one cluster's active set would split every cluster's sources
    // as finely, so cap the whole grid at 2^20 lanes (the size the autotuner
    // picks for one large block) by halving the split.  Autotuned shapes of a
    // batched context were measured on batched blocks and are kept.
    if (c.nc > 1 && c.pinned.lpi == 0) {
        if (!has_tuned(c, n_act_typ))
            while (L.split > 1 && n_act * L.lpi / L.ipt * L.split > (int64_t(1) << 20))
                L.split >>= 1;
        // a batched block with few active clusters: at least 2^16 lanes,
        // splitting further while every split keeps a tile of the largest
        const int64_t ns = n_src > 0 ? n_src : max_cluster(c);
        while (n_act * L.lpi / L.ipt * L.split < (int64_t(1) << 16) &&
               ns / ((int64_t)L.split * 2) >= 64 * L.waves &&
               (int64_t)L.split * 2 * n_act <= c.part_cap)
            L.split <<= 1;
    }
    const int64_t ib = iblock_size(L);
    ForceWork w{};
    w.idx = idx;
    w.seg = c.d_seg;
    w.off = c.d_off;
    w.split = L.split;
    w.nc = c.nc;
    w.err = c.d_err;
    if (c.nc == 1) {
        w.n_blocks = (n_act + ib - 1) / ib;
    } else {
        const int64_t cap = n_act / ib + c.nc + 1;
        HIPCHK(c, launch_blocks(c, ib, cap, c.stream));
        w.blk_cluster = c.d_blk_cluster;
        w.blk_first = c.d_blk_first;
        w.n_blocks = cap;
    }
    const size_t before = c.prof_pending.size();
    HIPCHK(c, launch_force(c, w, L, out, n_act, c.stream, reduce));
    if (used)
        *used = L;
    if (work)
        *work = w;
    // interactions of this launch, for the profile: n_act * N with one
    // cluster; with several, the block step fills it from the schedule
    for (size_t r = before; r < c.prof_pending.size(); ++r)
        if (c.prof_pending[r].phase == PH_FORCE)
            c.prof_pending[r].pairs = pairs_hint >= 0 ? pairs_hint : (double)n_act * (double)c.n;
    return NBODY_OK;
}

// the two start-up passes over every particle (see nbody_init)
int run_force_init(Ctx &c)
{
    hipStream_t s = c.stream;
    const int64_t n = c.n;
    HIPCHK(c, launch_segments(c, nullptr, n, s));
    Launch L = pick_launch(c, c.nc == 1 ? n : std::max<int64_t>(1, n / c.nc), max_cluster(c));
    L.split = 1;
    L.ipt = 1;   // the start-up kernels take one particle per lane group
    while (n * L.lpi < (int64_t(1) << 18) && L.lpi < 64)
        L.lpi <<= 1;
    const int64_t ib = iblock_size(L);
    ForceWork w{};
    w.seg = c.d_seg;
    w.off = c.d_off;
    w.split = 1;
    w.nc = c.nc;
    if (c.nc == 1) {
        w.n_blocks = (n + ib - 1) / ib;
    } else {
        const int64_t cap = n / ib + c.nc + 1;
        HIPCHK(c, launch_blocks(c, ib, cap, s));
        w.blk_cluster = c.d_blk_cluster;
        w.blk_first = c.d_blk_first;
        w.n_blocks = cap;
    }
    ForceOut o1{};
    o1.vec[0] = c.fnew;
    o1.vec[1] = c.fnew + 3 * n;
    o1.sk = 1;
    o1.sd = n;
    HIPCHK(c, launch_force_init(c, w, L, o1, s));
    HIPCHK(c, hipMemcpyAsync(c.st.acc, c.fnew, 3 * n * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c.st.jrk, c.fnew + 3 * n, 3 * n * 8, hipMemcpyDeviceToDevice, s));
    ForceOut o2{};
    o2.vec[2] = c.st.snp;
    o2.vec[3] = c.st.crk;
    o2.sk = 1;
    o2.sd = n;
    HIPCHK(c, launch_force_init(c, w, L, o2, s));
    return NBODY_OK;
}

// Waits until the kernel launched with sequence number seq has put its
// results into the mapped host words, by polling the sequence word (the
// kernel stores it after the results with system-scope release order);
// every 1024 polls the stream is queried, so that a failed or finished
// stream that never wrote the word ends the wait with an error instead of a
// hang.  After ~64 k polls (a long kernel, such as the device-resident loop)
// the host sleeps 20 us between polls instead of spinning.
int wait_words(Ctx &c, int first, int count, int seq_word, int64_t seq, int64_t *out)
{
    for (uint32_t spin = 1;; ++spin) {
        if (__atomic_load_n(&c.h_tot[seq_word], __ATOMIC_ACQUIRE) == seq)
            break;
        if (spin > (1u << 16))
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        if ((spin & 1023u) == 0) {
            const hipError_t e = hipStreamQuery(c.stream);
            if (e == hipSuccess) {
                if (__atomic_load_n(&c.h_tot[seq_word], __ATOMIC_ACQUIRE) == seq)
                    break;
                return fail(c, NBODY_EDEVICE, "a kernel did not report its totals");
            }
            if (e != hipErrorNotReady)
                return hip_fail(c, e, "block steps");
        }
        __builtin_ia32_pause();
    }
    for (int q = 0; q < count; ++q)
        out[q] = __atomic_load_n(&c.h_tot[first + q], __ATOMIC_RELAXED);
    return NBODY_OK;
}

int wait_totals(Ctx &c, int64_t seq, int64_t tot[6]) { return wait_words(c, 0, 6, 6, seq, tot); }

// Work split of the ensemble loop over G workgroups.  Cost model, in units
// of N^2 (pair evaluations per block step scale with N_c^2): a cluster on W
// workgroups costs N_c^2 / W + L_W, where L_W stands for the latency of its
// block steps (thousands of steps of a few barriers and memory round trips
// each, about the same count for every cluster of a King ensemble);
// measured on the 256-cluster King W0 = 6 ensemble on the MI355X: a
// one-workgroup cluster of 256 bodies takes as long as 6e5 N^2 units
// (~775^2), a multi-workgroup group about twice that.  The plan is the
// smallest makespan M (bisection) for which: a cluster with N_c^2 + L_1 > M
// gets a group of its own of ceil(N_c^2 / (M - L_W)) workgroups (at most
// ENS_GROUP_MAX), and the others are packed first-fit-decreasing onto
// single-workgroup groups of capacity M.  Workgroups left over go to the
// groups with the most work per workgroup.  A group integrates its clusters
// one after another.  Each group's partial slots are twice its largest
// cluster, so the groups' regions fit the split buffer (2 n slots).  Copies
// the tables to the device and sets c.ens; returns the number of workgroups
// to launch.
constexpr double ENS_LAT_ONE = 6.0e5, ENS_LAT_GROUP = 1.2e6;

int plan_ensemble(Ctx &c, int G)
{
    const int nc = c.nc;
    std::vector<int> order(nc);
    for (int k = 0; k < nc; ++k)
        order[k] = k;
    auto work = [&](int k) {
        const double s = (double)(c.off[k + 1] - c.off[k]);
        return s * s;
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
    double total = 0.0;
    for (int k = 0; k < nc; ++k)
        total += work(k);
    // groups for a makespan M: {clusters}, workgroups, work; false if they
    // need more than G workgroups or a cluster cannot finish within M
    std::vector<std::vector<int>> groups;
    std::vector<int> gsize;
    std::vector<double> gwork;
    auto build = [&](double M) {
        groups.clear();
        gsize.clear();
        gwork.clear();
        int used = 0;
        size_t q = 0;
        for (; q < order.size() && work(order[q]) + ENS_LAT_ONE > M; ++q) {
            const double w = work(order[q]);
            if (M <= ENS_LAT_GROUP)
                return false;
            const int W = (int)std::min<double>(std::ceil(w / (M - ENS_LAT_GROUP)),
                                                ENS_GROUP_MAX);
            if (w / W + ENS_LAT_GROUP > M * (1 + 1e-12))
                return false;
            groups.push_back({order[q]});
            gsize.push_back(W);
            gwork.push_back(w);
            used += W;
        }
        const size_t first_bin = groups.size();
        for (; q < order.size(); ++q) {
            const double w = work(order[q]) + ENS_LAT_ONE;
            size_t b = first_bin;
            while (b < groups.size() && gwork[b] + w > M * (1 + 1e-12))
                ++b;
            if (b == groups.size()) {
                groups.push_back({});
                gsize.push_back(1);
                gwork.push_back(0.0);
                ++used;
            }
            groups[b].push_back(order[q]);
            gwork[b] += w;
        }
        return used <= G;
    };
    double lo = total / G, hi = total + nc * (ENS_LAT_ONE + ENS_LAT_GROUP) + 1.0;
    for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (build(mid))
            hi = mid;
        else
            lo = mid;
    }
    if (!build(hi))
        return 0;
    int used = 0;
    for (int W : gsize)
        used += W;
    // spare workgroups to the groups with the most work per workgroup
    // (groups of one cluster only, so that a group's clusters keep sharing
    // one slice plan)
    for (; used < G; ++used) {
        int best = -1;
        double bw = 0.0;
        for (size_t g = 0; g < groups.size(); ++g)
            if (groups[g].size() == 1 && gsize[g] < ENS_GROUP_MAX && gwork[g] / gsize[g] > bw) {
                bw = gwork[g] / gsize[g];
                best = (int)g;
            }
        if (best < 0)
            break;
        ++gsize[best];
    }
    const int ng = (int)groups.size();
    if (ng > LOOP_GMAX)
        return 0;
    std::vector<int32_t> i32(4 * LOOP_GMAX + 1 + nc, 0);
    std::vector<int64_t> i64(4 * LOOP_GMAX, 0);
    int32_t *grp_of = i32.data(), *first = grp_of + LOOP_GMAX, *size = first + LOOP_GMAX;
    int32_t *cl_off = size + LOOP_GMAX, *cl = cl_off + LOOP_GMAX + 1;
    int64_t *part_off = i64.data(), *part_cap = part_off + LOOP_GMAX;
    int wg = 0, ncl = 0;
    int64_t slot = 0;
    for (int g = 0; g < ng; ++g) {
        first[g] = wg;
        size[g] = gsize[g];
        for (int k = 0; k < gsize[g]; ++k)
            grp_of[wg++] = g;
        cl_off[g] = ncl;
        int64_t big = 1;
        for (int k : groups[g]) {
            cl[ncl++] = k;
            big = std::max<int64_t>(big, c.off[k + 1] - c.off[k]);
        }
        part_off[g] = slot;
        part_cap[g] = 2 * big;
        slot += 2 * big;
    }
    cl_off[ng] = ncl;
    if (slot > c.part_cap || ncl != nc || wg > G)
        return 0;
    if (hipMemcpyAsync(c.d_ens_i32, i32.data(), i32.size() * 4, hipMemcpyHostToDevice,
                       c.stream) != hipSuccess ||
        hipMemcpyAsync(c.d_ens_i64, i64.data(), i64.size() * 8, hipMemcpyHostToDevice,
                       c.stream) != hipSuccess ||
        hipStreamSynchronize(c.stream) != hipSuccess)
        return 0;
    c.ens.grp_of = c.d_ens_i32;
    c.ens.first = c.d_ens_i32 + LOOP_GMAX;
    c.ens.size = c.d_ens_i32 + 2 * LOOP_GMAX;
    c.ens.cl_off = c.d_ens_i32 + 3 * LOOP_GMAX;
    c.ens.cl = c.d_ens_i32 + 4 * LOOP_GMAX + 1;
    c.ens.part_off = c.d_ens_i64;
    c.ens.part_cap = c.d_ens_i64 + LOOP_GMAX;
    c.ens.seg = c.d_ens_i64 + 2 * LOOP_GMAX;
    return wg;
}

// A batched context's block steps to t_target in one launch (the ensemble
// loop); *done = false when the loop is not used (then the host-sized path
// runs the steps).
int run_ensemble(Ctx &c, double t_target, nbody_step_stats *stats, bool *done)
{
    *done = false;
    if (c.nc <= 1 || c.loop_amax == 0 || c.pinned.lpi != 0 || c.prof)
        return NBODY_OK;
    if (c.ens_grid < 0) {
        const int G = ensemble_max_grid(c);
        c.ens_grid = G >= 1 ? plan_ensemble(c, G) : 0;
    }
    if (c.ens_grid <= 0)
        return NBODY_OK;
    // barrier lines of the workgroups, then the groups' unit counters
    HIPCHK(c, hipMemsetAsync(c.d_loop_bar, 0, 2 * LOOP_BAR_WORDS * sizeof(uint32_t), c.stream));
    HIPCHK(c, hipMemsetAsync(c.d_ens_res, 0, 4 * 8, c.stream));
    if (launch_ensemble_loop(c, t_target, c.ens_grid, c.ens, c.d_ens_res, c.stream) !=
        hipSuccess) {
        // the runtime refused the cooperative launch (nothing was enqueued):
        // clear that error and keep to the host-sized path from now on
        (void)hipGetLastError();
        c.ens_grid = 0;
        return NBODY_OK;
    }
    unsigned long long r[4];
    HIPCHK(c, hipMemcpyAsync(r, c.d_ens_res, 4 * 8, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(c, hipStreamSynchronize(c.stream));
    if (stats) {
        stats->block_steps += (int64_t)r[2];
        stats->active_total += (int64_t)r[0];
        stats->interactions += (double)r[1];
    }
    if (int rc = take_err(c))
        return rc;
    *done = true;
    return NBODY_OK;
}

// Block steps inside one cooperative launch while the active sets stay at
// or below the loop's limit (one system, no pinned shape, no profiling).
// Measured on MI355X: a grid barrier costs a few microseconds and grows
// with the number of workgroups, and the loop's few workgroups evaluate a
// large block at low occupancy, so the loop uses 64 workgroups, takes blocks
// of up to ~2^21 pairs, and is switched on automatically for systems of up
// to 4096 bodies only (there it cuts the time per block step by 7-15 %
// against the host-sized path with its schedule from per-level counts; at
// 6144 bodies and beyond it is slower).
// *reason: LOOP_DONE (every particle at the target), LOOP_BIG (the next
// block is larger than the limit: the host path takes it) or 0 when the
// loop is not used.
int run_loop(Ctx &c, double t_target, nbody_step_stats *stats, int *reason)
{
    *reason = 0;
    if (c.nc != 1 || c.loop_amax == 0 || c.pinned.lpi != 0 || c.prof)
        return NBODY_OK;
    if (c.loop_amax < 0 && c.n > LOOP_AUTO_NMAX)
        return NBODY_OK;
    if (c.loop_grid < 0)
        c.loop_grid = std::min(step_loop_max_grid(c), LOOP_GRID);
    if (c.loop_grid <= 0)
        return NBODY_OK;
    // automatic limit: blocks of up to ~2^21 pairs, at least 4 particles,
    // within the split partials' capacity at the loop's largest split
    int64_t a_max = c.loop_amax;
    if (a_max < 0) {
        a_max = 4;
        while (a_max * 2 * c.n <= (int64_t(1) << 21))
            a_max *= 2;
    }
    a_max = std::min<int64_t>(a_max, c.part_cap / 64);
    HIPCHK(c, hipMemsetAsync(c.d_loop_bar, 0, 32 * c.loop_grid * sizeof(uint32_t), c.stream));
    const int64_t seq = ++c.loop_seq;
    if (launch_step_loop(c, t_target, a_max, c.loop_grid, seq, c.stream) != hipSuccess) {
        // the runtime refused the cooperative launch (nothing was enqueued):
        // clear that error and keep to the host-sized path from now on
        (void)hipGetLastError();
        c.loop_grid = 0;
        return NBODY_OK;
    }
    int64_t r[5];
    if (int rc = wait_words(c, 8, 5, 15, seq, r))
        return rc;
    if (stats) {
        stats->block_steps += r[0];
        stats->active_total += r[1];
        stats->interactions += (double)r[2];
    }
    if (r[3] == LOOP_ERR)
        return take_err(c);
    *reason = (int)r[3];
    return NBODY_OK;
}

// Whether nbody_step schedules this context from per-level counts: one
// system, not left to the device-resident loop, a level range that fits
// LVL_N, and a state that meets the conditions (every step a power of two in
// [dt_min, dt_max], every particle at a multiple of its step and short of its
// next one); the counts are built here, once per call.
int levels_ready(Ctx &c, bool *ok)
{
    *ok = false;
    if (c.nc != 1 || c.sched_mode != 0)
        return NBODY_OK;
    const bool loop = c.loop_amax != 0 && c.pinned.lpi == 0 && !c.prof && c.loop_grid != 0 &&
                      !(c.loop_amax < 0 && c.n > LOOP_AUTO_NMAX);
    if (loop || std::ilogb(c.cfg.dt_max) - std::ilogb(c.cfg.dt_min) >= LVL_N)
        return NBODY_OK;
    HIPCHK(c, launch_levels_build(c, c.stream));
    HIPCHK(c, hipMemcpyAsync(c.h_info, c.d_lvl + LVL_BAD, sizeof(int64_t), hipMemcpyDeviceToHost,
                             c.stream));
    HIPCHK(c, hipStreamSynchronize(c.stream));
    *ok = c.h_info[0] == 0;
    return NBODY_OK;
}

// one block step; fills n_act / t_block and adds to stats.  levels: the
// schedule comes from the per-level counts (levels_ready said so), which
// the corrector keeps up to date
int block_step(Ctx &c, double t_target, int64_t *n_act_out, double *t_block_out,
               nbody_step_stats *stats, bool levels)
{
    // the host needs N_act (and the block time) to size the evaluation; it
    // waits for the scan's totals only (written into mapped host memory),
    // while the GPU goes on with the compaction of the active list and the
    // predictor (which skips clusters past the target, so it is harmless
    // when nothing is due)
    int rec = prof_begin(c, PH_SCHED);
    const int64_t seq = ++c.sched_seq;
    if (levels)
        HIPCHK(c, launch_levels_sched(c, t_target, seq, c.stream));
    else
        HIPCHK(c, launch_sched_head(c, t_target, seq, c.stream));
    prof_end(c, rec);
    rec = prof_begin(c, PH_PREDICT);   // the compaction of the active list runs here too
    HIPCHK(c, launch_scatter_pack(c, c.stream, levels));
    prof_end(c, rec);
    int64_t tot[6];
    if (int rc = wait_totals(c, seq, tot))
        return rc;
    const int64_t n_act = tot[0];
    double tb;
    std::memcpy(&tb, &tot[1], 8);
    if (tot[3] != 0)
        return take_err(c);
    *n_act_out = n_act;
    *t_block_out = tb;
    if (n_act == 0)
        return NBODY_OK;
    ForceOut out{};
    out.vec[0] = c.fnew;
    out.vec[1] = c.fnew + 3 * n_act;
    out.vec[2] = c.fnew + 6 * n_act;
    out.pot = nullptr;
    out.sk = 1;
    out.sd = n_act;
    // launch shape from the typical active set of the clusters that have
    // one, against the largest of them
    const int64_t typ = c.nc == 1 ? n_act : std::max<int64_t>(1, n_act / std::max<int64_t>(1, tot[4]));
    // with a split, the reduction of the partials is fused into the corrector
    Launch L;
    ForceWork w;
    int rc = run_force(c, c.act, n_act, typ, out, (double)tot[2], tot[5], false, &L, &w);
    if (rc)
        return rc;
    rec = prof_begin(c, PH_CORRECT);
    if (w.split > 1)
        HIPCHK(c, launch_reduce_correct(c, w, w.split, 64 * L.waves, n_act, t_target, c.stream,
                                        levels));
    else
        HIPCHK(c, launch_correct(c, n_act, c.act, t_target, out.vec[0], out.vec[1], out.vec[2], 1,
                                 n_act, c.stream, levels));
    prof_end(c, rec);
    if (stats) {
        stats->block_steps += 1;
        stats->active_total += n_act;
        stats->interactions += (double)tot[2];
    }
    return NBODY_OK;
}

bool on_grid(double t, double dt_min)
{
    if (!(t >= 0.0) || !std::isfinite(t))
        return false;
    const double q = t / dt_min;
    return q == std::floor(q);
}

}  // namespace

extern "C" {

void nbody_default_config(nbody_config *cfg)
{
    if (!cfg)
        return;
    std::memset(cfg, 0, sizeof *cfg);
    cfg->eta = 0.45;
    cfg->eta_init = 0.1;
    cfg->dt_min = std::ldexp(1.0, -25);
    cfg->dt_max = 1.0 / 16;
    cfg->precision = NBODY_PREC_MIXED;
    cfg->n_clusters = 1;
}

size_t nbody_workspace_bytes(int64_t n, const nbody_config *cfg)
{
    if (n <= 0 || n > (int64_t(1) << 31) - 1 || !config_ok(cfg, n))
        return 0;
    return (size_t)ws_layout(n, n_clusters(cfg), cfg->precision, nullptr, nullptr);
}

const char *nbody_strerror(int code)
{
    switch (code) {
    case NBODY_OK: return "ok";
    case NBODY_EINVAL: return "invalid argument";
    case NBODY_EDEVICE: return "HIP runtime error";
    case NBODY_ENONFINITE: return "non-finite value";
    case NBODY_EDTMIN: return "time step below dt_min required";
    case NBODY_ESTATE: return "invalid state for this call";
    default: return "unknown error";
    }
}

const char *nbody_last_error(const nbody_ctx *ctx)
{
    return ctx ? ctx->c.last_error.c_str() : "null context";
}

int nbody_init(nbody_ctx **out, int64_t n, const double *d_mass, const double *d_pos,
               const double *d_vel, double eps, const nbody_config *cfg, void *d_workspace,
               size_t ws_bytes)
{
    if (!out)
        return NBODY_EINVAL;
    *out = nullptr;
    if (n <= 0 || n > (int64_t(1) << 31) - 1 || !d_mass || !d_pos || !d_vel || !d_workspace ||
        !(eps >= 0.0) || !std::isfinite(eps) || !config_ok(cfg, n))
        return NBODY_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_workspace) % ALIGN) != 0)
        return NBODY_EINVAL;
    const int32_t nc = n_clusters(cfg);
    if ((int64_t)ws_bytes < ws_layout(n, nc, cfg->precision, nullptr, nullptr))
        return NBODY_EINVAL;
    nbody_ctx *h = new (std::nothrow) nbody_ctx;
    if (!h)
        return NBODY_EINVAL;
    Ctx &c = h->c;
    c.n = n;
    c.nc = nc;
    c.eps = eps;
    c.cfg = *cfg;
    c.cfg.cluster_offsets = nullptr;
    c.stream = (hipStream_t)cfg->stream;
    auto bail = [&](int rc) {
        if (c.h_tot)
            (void)hipHostFree(c.h_tot);
        if (c.h_info)
            (void)hipHostFree(c.h_info);
        delete h;
        return rc;
    };
    if (hipGetDevice(&c.device) != hipSuccess)
        return bail(NBODY_EDEVICE);
    ws_layout(n, nc, cfg->precision, &c, static_cast<char *>(d_workspace));
    if (hipHostMalloc((void **)&c.h_info, 64 * sizeof(int64_t) + 64 * sizeof(double) + 64,
                      hipHostMallocDefault) != hipSuccess)
        return bail(NBODY_EDEVICE);
    c.h_red = reinterpret_cast<double *>(c.h_info + 64);
    c.h_err = reinterpret_cast<uint32_t *>(c.h_red + 64);
    if (hipHostMalloc((void **)&c.h_tot, 16 * sizeof(int64_t),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer((void **)&c.d_tot, c.h_tot, 0) != hipSuccess)
        return bail(NBODY_EDEVICE);
    std::memset(c.h_tot, 0, 16 * sizeof(int64_t));
    // cluster offsets, cluster of each particle, schedule chunk table
    c.off.assign(nc + 1, 0);
    if (nc > 1)
        std::copy(cfg->cluster_offsets, cfg->cluster_offsets + nc + 1, c.off.begin());
    else
        c.off[1] = n;
    std::vector<int32_t> ch_cl;
    std::vector<int64_t> ch_b;
    for (int32_t k = 0; k < nc; ++k)
        for (int64_t b = c.off[k]; b < c.off[k + 1]; b += SCHED_CHUNK) {
            ch_cl.push_back(k);
            ch_b.push_back(b);
        }
    ch_b.push_back(n);
    c.n_chunks = (int64_t)ch_cl.size();
    hipStream_t s = c.stream;
    int rc = NBODY_OK;
    auto H = [&](hipError_t e, const char *w) {
        if (e != hipSuccess && rc == NBODY_OK)
            rc = hip_fail(c, e, w);
    };
    H(hipMemcpyAsync(c.d_off, c.off.data(), (nc + 1) * 8, hipMemcpyHostToDevice, s), "offsets");
    H(hipMemcpyAsync(c.d_chunk_cluster, ch_cl.data(), c.n_chunks * 4, hipMemcpyHostToDevice, s), "chunks");
    H(hipMemcpyAsync(c.d_chunk_begin, ch_b.data(), (c.n_chunks + 1) * 8, hipMemcpyHostToDevice, s), "chunks");
    if (nc > 1) {
        std::vector<int32_t> cl(n);
        for (int32_t k = 0; k < nc; ++k)
            std::fill(cl.begin() + c.off[k], cl.begin() + c.off[k + 1], k);
        H(hipMemcpyAsync(c.d_cluster_of, cl.data(), n * 4, hipMemcpyHostToDevice, s), "cluster_of");
        H(hipStreamSynchronize(s), "sync");   // host vectors go out of scope
    }
    H(hipMemsetAsync(c.d_err, 0, 4, s), "err");
    H(hipMemsetAsync(c.d_info, 0, 64 * 8, s), "info");
    H(launch_sched_reset(c, s), "sched");   // the scan keeps them reset afterwards
    H(hipMemcpyAsync(c.st.mass, d_mass, n * 8, hipMemcpyDeviceToDevice, s), "mass");
    H(launch_aos_to_soa(d_pos, c.st.pos, n, s), "pos");
    H(launch_aos_to_soa(d_vel, c.st.vel, n, s), "vel");
    H(hipMemsetAsync(c.st.acc, 0, 3 * n * 8, s), "acc");
    H(hipMemsetAsync(c.st.jrk, 0, 3 * n * 8, s), "jrk");
    H(hipMemsetAsync(c.st.snp, 0, 3 * n * 8, s), "snp");
    H(hipMemsetAsync(c.st.crk, 0, 3 * n * 8, s), "crk");
    H(hipMemsetAsync(c.st.t, 0, n * 8, s), "t");
    H(launch_check_finite(c, s), "finite");
    H(hipStreamSynchronize(s), "sync");
    if (rc != NBODY_OK)
        return bail(rc);
    rc = take_err(c);
    if (rc != NBODY_OK)
        return bail(rc);
    // start-up evaluation, FP64 from the stored state: pass 1 gives a and da
    // (the sources' zero a and da do not enter them); pass 2 gives d2a and
    // the crackle with the pass-1 values as the sources' a and da.  Then the
    // first steps.
    if (!cfg->skip_startup) {
        if (rc == NBODY_OK)
            rc = run_force_init(c);
        H(launch_init_dt(c, s), "init_dt");
    } else {
        H(launch_init_dt(c, s), "init_dt");   // zero derivatives: dt = dt_max
    }
    if (rc == NBODY_OK)
        rc = take_err(c);
    if (rc != NBODY_OK)
        return bail(rc);
    *out = h;
    return NBODY_OK;
}

void nbody_free(nbody_ctx *ctx)
{
    if (!ctx)
        return;
    // kernels still queued on the stream may write the mapped host words
    (void)hipStreamSynchronize(ctx->c.stream);
    (void)prof_collect(ctx->c);
    for (hipEvent_t e : ctx->c.prof_pool)
        (void)hipEventDestroy(e);
    if (ctx->c.h_tot)
        (void)hipHostFree(ctx->c.h_tot);
    if (ctx->c.h_info)
        (void)hipHostFree(ctx->c.h_info);
    delete ctx;
}

int nbody_force(nbody_ctx *ctx, int64_t n_act, const int32_t *d_idx, double *d_acc,
                double *d_jrk, double *d_snp, double *d_pot)
{
    if (!ctx)
        return NBODY_EINVAL;
    Ctx &c = ctx->c;
    if (n_act < 0 || n_act > c.n)
        return fail(c, NBODY_EINVAL, "n_act out of range");
    if (n_act == 0)
        return NBODY_OK;
    if (!d_idx || !d_acc || !d_jrk || !d_snp)
        return fail(c, NBODY_EINVAL, "null pointer");
    if (c.cfg.validate) {
        HIPCHK(c, launch_validate_idx(c, n_act, d_idx, c.stream));
        const int rc = take_err(c);
        if (rc)
            return rc;
    }
    HIPCHK(c, launch_pack(c, nullptr, 1, nullptr, c.stream));
    HIPCHK(c, launch_segments(c, d_idx, n_act, c.stream));
    ForceOut out{};
    out.vec[0] = d_acc;
    out.vec[1] = d_jrk;
    out.vec[2] = d_snp;
    out.pot = d_pot;
    out.sk = 3;
    out.sd = 1;
    const int64_t typ = c.nc == 1 ? n_act : std::max<int64_t>(1, n_act / c.nc);
    return run_force(c, d_idx, n_act, typ, out, c.nc == 1 ? (double)n_act * (double)c.n : 0.0);
}

int nbody_predict(nbody_ctx *ctx, double t, double *d_pos, double *d_vel, double *d_acc)
{
    if (!ctx)
        return NBODY_EINVAL;
    Ctx &c = ctx->c;
    if (!d_pos || !d_vel || !d_acc || !std::isfinite(t))
        return fail(c, NBODY_EINVAL, "bad argument");
    HIPCHK(c, launch_predict_out(c, t, d_pos, d_vel, d_acc, c.stream));
    return NBODY_OK;
}

int nbody_schedule(nbody_ctx *ctx, double t_target, int32_t *d_idx, int64_t *n_act,
                   double *t_next)
{
    if (!ctx)
        return NBODY_EINVAL;
    Ctx &c = ctx->c;
    if (!d_idx || !n_act || !t_next || !on_grid(t_target, c.cfg.dt_min))
        return fail(c, NBODY_EINVAL, "bad argument");
    HIPCHK(c, launch_schedule(c, t_target, ++c.sched_seq, c.stream));
    HIPCHK(c, hipMemcpyAsync(c.h_info, c.d_info, 8 * sizeof(int64_t), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(c, hipStreamSynchronize(c.stream));
    *n_act = c.h_info[0];
    std::memcpy(t_next, &c.h_info[1], 8);
    if (*n_act > 0)
        HIPCHK(c, hipMemcpyAsync(d_idx, c.act, *n_act * 4, hipMemcpyDeviceToDevice, c.stream));
    HIPCHK(c, hipStreamSynchronize(c.stream));
    return NBODY_OK;
}

int nbody_correct(nbody_ctx *ctx, int64_t n_act, const int32_t *d_idx, double t_target,
                  const double *d_acc, const double *d_jrk, const double *d_snp)
{
    if (!ctx)
        return NBODY_EINVAL;
    Ctx &c = ctx->c;
    if (n_act < 0 || n_act > c.n || (n_act > 0 && (!d_idx || !d_acc || !d_jrk || !d_snp)) ||
        !on_grid(t_target, c.cfg.dt_min))
        return fail(c, NBODY_EINVAL, "bad argument");
    if (c.cfg.validate && n_act > 0) {
        HIPCHK(c, launch_validate_idx(c, n_act, d_idx, c.stream));
        const int rc = take_err(c);
        if (rc)
            return rc;
    }
    HIPCHK(c, launch_correct(c, n_act, d_idx, t_target, d_acc, d_jrk, d_snp, 3, 1, c.stream));
    return take_err(c);
}

int nbody_block_step(nbody_ctx *ctx, double t_target, int64_t *n_act, double *t_block)
{
    if (!ctx)
        return NBODY_EINVAL;
    Ctx &c = ctx->c;
    if (!n_act || !t_block || !on_grid(t_target, c.cfg.dt_min))
        return fail(c, NBODY_EINVAL, "bad argument");
    int rc = block_step(c, t_target, n_act, t_block, nullptr, false);
    if (rc)
        return rc;
    return take_err(c);
}

int nbody_step(nbody_ctx *ctx, double t_target, nbody_step_stats *stats)
{
    if (!ctx)
        return NBODY_EINVAL;
    Ctx &c = ctx->c;
    if (!on_grid(t_target, c.cfg.dt_min))
        return fail(c, NBODY_EINVAL, "t_target not a non-negative multiple of dt_min");
    if (stats)
        std::memset(stats, 0, sizeof *stats);
    HIPCHK(c, hipMemsetAsync(c.d_info + 8, 0, 40 * 8, c.stream));
    HIPCHK(c, launch_recap(c, t_target, c.stream));
    int rc = take_err(c);
    if (rc)
        return rc;
    // independent clusters: every block step in one launch
    bool done = false;
    rc = run_ensemble(c, t_target, stats, &done);
    if (rc)
        return rc;
    bool levels = false;
    if (!done && (rc = levels_ready(c, &levels)) != NBODY_OK)
        return rc;
    for (; !done;) {
        // small blocks inside one launch; a larger one on the host path
        int reason = 0;
        rc = run_loop(c, t_target, stats, &reason);
        if (rc)
            return rc;
        if (reason == LOOP_DONE)
            break;
        int64_t na = 0;
        double tb = 0.0;
        rc = block_step(c, t_target, &na, &tb, stats, levels);
        if (rc)
            return rc;
        if (na == 0)
            break;
    }
    if (stats) {
        HIPCHK(c, hipMemcpyAsync(c.h_info + 8, c.d_info + 8, 40 * 8, hipMemcpyDeviceToHost, c.stream));
        HIPCHK(c, hipStreamSynchronize(c.stream));
        for (int b = 0; b < 40; ++b)
            stats->hist[b] = c.h_info[8 + b];
    }
    return take_err(c);
}

int nbody_get_state(nbody_ctx *ctx, double *d_pos, double *d_vel, double *d_acc, double *d_jrk,
                    double *d_snp, double *d_crk, double *d_t, double *d_dt)
{
    if (!ctx)
        return NBODY_EINVAL;
    Ctx &c = ctx->c;
    const double *src[6] = {c.st.pos, c.st.vel, c.st.acc, c.st.jrk, c.st.snp, c.st.crk};
    double *dst[6] = {d_pos, d_vel, d_acc, d_jrk, d_snp, d_crk};
    for (int q = 0; q < 6; ++q)
        if (dst[q])
            HIPCHK(c, launch_soa_to_aos(src[q], dst[q], c.n, c.stream));
    if (d_t)
        HIPCHK(c, hipMemcpyAsync(d_t, c.st.t, c.n * 8, hipMemcpyDeviceToDevice, c.stream));
    if (d_dt)
        HIPCHK(c, hipMemcpyAsync(d_dt, c.st.dt, c.n * 8, hipMemcpyDeviceToDevice, c.stream));
    return NBODY_OK;
}

int nbody_set_state(nbody_ctx *ctx, const double *d_pos, const double *d_vel,
                    const double *d_acc, const double *d_jrk, const double *d_snp,
                    const double *d_crk, const double *d_t, const double *d_dt)
{
    if (!ctx)
        return NBODY_EINVAL;
    Ctx &c = ctx->c;
    const double *src[6] = {d_pos, d_vel, d_acc, d_jrk, d_snp, d_crk};
    double *dst[6] = {c.st.pos, c.st.vel, c.st.acc, c.st.jrk, c.st.snp, c.st.crk};
    for (int q = 0; q < 6; ++q)
        if (src[q])
            HIPCHK(c, launch_aos_to_soa(src[q], dst[q], c.n, c.stream));
    if (d_t)
        HIPCHK(c, hipMemcpyAsync(c.st.t, d_t, c.n * 8, hipMemcpyDeviceToDevice, c.stream));
    if (d_dt)
        HIPCHK(c, hipMemcpyAsync(c.st.dt, d_dt, c.n * 8, hipMemcpyDeviceToDevice, c.stream));
    return NBODY_OK;
}

int nbody_energy(nbody_ctx *ctx, double *ekin, double *epot, double L[3])
{
    if (!ctx)
        return NBODY_EINVAL;
    Ctx &c = ctx->c;
    HIPCHK(c, launch_sync_check(c, c.stream));
    const int rc = take_err(c);
    if (rc)
        return rc;
    HIPCHK(c, launch_energy_pot(c, c.d_phi, c.stream));
    const int rec = prof_begin(c, PH_ENERGY);
    HIPCHK(c, launch_energy_sums(c, c.d_phi, c.d_red + c.red_cap - 8, c.stream));
    prof_end(c, rec);
    HIPCHK(c, hipMemcpyAsync(c.h_red, c.d_red + c.red_cap - 8, 5 * 8, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(c, hipStreamSynchronize(c.stream));
    if (ekin)
        *ekin = c.h_red[0];
    if (epot)
        *epot = c.h_red[1];
    if (L) {
        L[0] = c.h_red[2];
        L[1] = c.h_red[3];
        L[2] = c.h_red[4];
    }
    return NBODY_OK;
}

int nbody_set_launch(nbody_ctx *ctx, const nbody_launch *shape)
{
    if (!ctx || !shape)
        return NBODY_EINVAL;
    Ctx &c = ctx->c;
    if (shape->lanes_per_i == 0 || shape->waves == 0 || shape->split == 0) {
        c.pinned = Launch{};
        return NBODY_OK;
    }
    const int l = shape->lanes_per_i;
    const int ipt = shape->i_per_lane == 0 ? 1 : shape->i_per_lane;
    if (l < 1 || l > 64 || (l & (l - 1)) || (shape->waves != 1 && shape->waves != 2 &&
                                             shape->waves != 4) || shape->split < 1 ||
        shape->split > 65535 || ipt < 1 || ipt > 2 || (ipt == 2 && l > 4))
        return fail(c, NBODY_EINVAL, "bad launch shape");
    c.pinned.lpi = l;
    c.pinned.waves = shape->waves;
    c.pinned.split = shape->split;
    c.pinned.ipt = ipt;
    return NBODY_OK;
}

int nbody_get_tuning(nbody_ctx *ctx, nbody_launch *table, int32_t max)
{
    if (!ctx || max < 0 || (max > 0 && !table))
        return NBODY_EINVAL;
    const Ctx &c = ctx->c;
    const int32_t cnt = (int32_t)c.tuned.size();
    for (int32_t b = 0; b < std::min(cnt, max); ++b) {
        table[b].lanes_per_i = c.tuned[b].lpi;
        table[b].waves = c.tuned[b].waves;
        table[b].split = c.tuned[b].split;
        table[b].i_per_lane = c.tuned[b].lpi > 0 ? c.tuned[b].ipt : 0;
    }
    return cnt;
}

int nbody_set_tuning(nbody_ctx *ctx, const nbody_launch *table, int32_t count)
{
    if (!ctx || count < 0 || count > 40 || (count > 0 && !table))
        return NBODY_EINVAL;
    Ctx &c = ctx->c;
    std::vector<Launch> t(count);
    for (int32_t b = 0; b < count; ++b) {
        const nbody_launch &e = table[b];
        if (e.lanes_per_i == 0 && e.waves == 0 && e.split == 0)
            continue;   // no tuned shape for this size
        const int l = e.lanes_per_i;
        const int ipt = e.i_per_lane == 0 ? 1 : e.i_per_lane;
        if (l < 1 || l > 64 || (l & (l - 1)) || (e.waves != 1 && e.waves != 2 && e.waves != 4) ||
            e.split < 1 || e.split > 65535 || ipt < 1 || ipt > 2 || (ipt == 2 && l > 4))
            return fail(c, NBODY_EINVAL, "bad launch shape in the tuning table");
        t[b].lpi = l;
        t[b].waves = e.waves;
        t[b].split = e.split;
        t[b].ipt = ipt;
    }
    c.tuned = t;
    return NBODY_OK;
}

int nbody_set_step_loop(nbody_ctx *ctx, int64_t max_active)
{
    if (!ctx)
        return NBODY_EINVAL;
    ctx->c.loop_amax = max_active < 0 ? -1 : max_active;
    return NBODY_OK;
}

int nbody_set_schedule(nbody_ctx *ctx, int mode)
{
    if (!ctx || (mode != 0 && mode != 1))
        return NBODY_EINVAL;
    ctx->c.sched_mode = mode;
    return NBODY_OK;
}

int nbody_get_launch(nbody_ctx *ctx, int64_t n_act, nbody_launch *shape)
{
    if (!ctx || !shape || n_act < 1)
        return NBODY_EINVAL;
    Ctx &c = ctx->c;
    Launch L = pick_launch(c, n_act, max_cluster(c));
    while ((int64_t)L.split * n_act > c.part_cap && L.split > 1)
        L.split >>= 1;
    shape->lanes_per_i = L.lpi;
    shape->waves = L.waves;
    shape->split = L.split;
    shape->i_per_lane = L.ipt;
    return NBODY_OK;
}

int nbody_autotune(nbody_ctx *ctx, double max_ms)
{
    if (!ctx)
        return NBODY_EINVAL;
    Ctx &c = ctx->c;
    if (!(max_ms > 0.0))
        max_ms = 200.0;
    const int64_t nsrc = max_cluster(c);
    size_t big = 0;
    for (size_t k = 0; k + 1 < c.off.size(); ++k)
        if (c.off[k + 1] - c.off[k] == nsrc) {
            big = k;
            break;
        }
    hipStream_t s = c.stream;
    // sources = the stored state; outputs to the integrator's scratch
    HIPCHK(c, launch_pack(c, nullptr, 1, nullptr, s));
    const bool was_prof = c.prof;
    c.prof = false;
    const Launch pinned = c.pinned;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    std::vector<Launch> table;
    int rc = NBODY_OK;
    std::vector<int32_t> hidx;
    // per size na (a power of two): one system takes na evenly spread
    // particles; a batched context takes up to na particles of every cluster,
    // the block a batched step with typical active set na looks like.  Sizes
    // whose single launch stays below ~2^35 pairs (tens of ms); larger active
    // sets keep the launch rule, which is then saturating anyway.
    for (int b = 0; rc == NBODY_OK && (int64_t(1) << b) <= nsrc; ++b) {
        const int64_t na = int64_t(1) << b;
        hidx.clear();
        double pairs = 0.0;
        for (size_t q = (c.nc > 1 ? 0 : big); q + 1 < c.off.size(); ++q) {
            const int64_t size = c.off[q + 1] - c.off[q];
            const int64_t cnt = std::min(na, size);
            for (int64_t k = 0; k < cnt; ++k)
                hidx.push_back((int32_t)(c.off[q] + k * size / cnt));
            pairs += (double)cnt * (double)size;
            if (c.nc == 1)
                break;
        }
        if (pairs > std::ldexp(1.0, 35))
            break;
        const int64_t nt = (int64_t)hidx.size();
        if (hipMemcpyAsync(c.act, hidx.data(), nt * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = hip_fail(c, hipGetLastError(), "autotune copy");
            break;
        }
        if (launch_segments(c, c.act, nt, s) != hipSuccess) {
            rc = hip_fail(c, hipGetLastError(), "autotune segments");
            break;
        }
        ForceOut out{};
        out.vec[0] = c.fnew;
        out.vec[1] = c.fnew + 3 * nt;
        out.vec[2] = c.fnew + 6 * nt;
        out.sk = 1;
        out.sd = nt;
        Launch best{};
        float best_ms = 1e30f;
        double spent = 0.0;
        for (int waves : {4, 2, 1}) {
            for (int lpi = 1; lpi <= 64; lpi <<= 1) {
              for (int ipt = 1; ipt <= (lpi <= 4 ? 2 : 1); ++ipt) {
                for (int split = 1; split <= 4096; split <<= 1) {
                    const int64_t lanes = nt * lpi * split / ipt;
                    if (lanes < (int64_t(1) << 14) && !(lpi == 64 && split >= nsrc / (64 * waves)))
                        continue;   // too little parallelism (unless nothing more is possible)
                    if (lanes > (int64_t(1) << 22) || split * nt > c.part_cap)
                        continue;
                    if (split > 1 && nsrc / split < 64 * waves)
                        continue;   // less than one tile per split
                    if (64 * waves > 64 * 4 || na * lpi < 64 * waves / 4)
                        continue;   // mostly idle workgroups
                    c.pinned.lpi = lpi;
                    c.pinned.waves = waves;
                    c.pinned.split = split;
                    c.pinned.ipt = ipt;
                    // one warm-up, then the minimum of 2 timed launches (of 6 when
                    // a launch is shorter than 0.2 ms, where timing noise is
                    // comparable to the differences between shapes)
                    float ms = 0.0f;
                    bool ok = true;
                    for (int rep = 0, reps = 3; rep < reps && ok; ++rep) {
                        ok = hipEventRecord(e0, s) == hipSuccess;
                        ok = ok && run_force(c, c.act, nt, na, out) == NBODY_OK;
                        ok = ok && hipEventRecord(e1, s) == hipSuccess;
                        ok = ok && hipEventSynchronize(e1) == hipSuccess;
                        float t = 0.0f;
                        ok = ok && hipEventElapsedTime(&t, e0, e1) == hipSuccess;
                        if (rep > 0)
                            ms = rep == 1 ? t : std::min(ms, t);
                        if (rep == 1 && t < 0.2f)
                            reps = 7;
                        spent += t;
                    }
                    if (!ok) {
                        rc = hip_fail(c, hipGetLastError(), "autotune launch");
                        break;
                    }
                    if (ms < best_ms) {
                        best_ms = ms;
                        best = c.pinned;
                    }
                    if (spent > max_ms)
                        break;
                }
                if (rc || spent > max_ms)
                    break;
              }
              if (rc || spent > max_ms)
                  break;
            }
            if (rc || spent > max_ms)
                break;
        }
        table.push_back(best);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c.pinned = pinned;
    c.prof = was_prof;
    if (rc == NBODY_OK)
        c.tuned = table;
    return rc;
}

int nbody_profile(nbody_ctx *ctx, int enable, nbody_profile_times *out)
{
    if (!ctx)
        return NBODY_EINVAL;
    Ctx &c = ctx->c;
    HIPCHK(c, prof_collect(c));
    if (out) {
        for (int p = 0; p < NBODY_NPHASE; ++p) {
            out->ms[p] = c.prof_ms[p];
            out->launches[p] = c.prof_cnt[p];
        }
        out->pairs = c.prof_pairs;
    }
    if (enable && !c.prof) {
        for (int p = 0; p < PH_N; ++p) {
            c.prof_ms[p] = 0.0;
            c.prof_cnt[p] = 0;
        }
        c.prof_pairs = 0.0;
        c.flog_nact.clear();
        c.flog_pairs.clear();
        c.flog_ms.clear();
    }
    c.prof = enable != 0;
    return NBODY_OK;
}

int nbody_force_noalloc(int64_t n, const double *d_mass, const double *d_pos,
                        const double *d_vel, const double *d_acc, double eps, int32_t precision,
                        int64_t n_act, const int32_t *d_idx, double *d_acc_out,
                        double *d_jrk_out, double *d_snp_out, double *d_pot_out, void *stream)
{
    if (n <= 0 || n > (int64_t(1) << 31) - 1 || n_act < 0 || n_act > n || !(eps >= 0.0) ||
        !std::isfinite(eps) ||
        (precision != NBODY_PREC_MIXED && precision != NBODY_PREC_FP64 &&
         precision != NBODY_PREC_FP32PAIR))
        return NBODY_EINVAL;
    if (n_act == 0)
        return NBODY_OK;
    if (!d_mass || !d_pos || !d_vel || !d_acc || !d_idx || !d_acc_out || !d_jrk_out ||
        !d_snp_out)
        return NBODY_EINVAL;
    // host-side description of the evaluation: no workspace, no state
    Ctx c;
    c.n = n;
    c.nc = 1;
    c.eps = eps;
    nbody_default_config(&c.cfg);
    c.cfg.precision = precision;
    c.cfg.stream = stream;
    c.stream = (hipStream_t)stream;
    int64_t *seg = nullptr, *off = nullptr;
    const int64_t head = noalloc_layout(n, precision, &c, nullptr, &seg, &off);
    const int64_t cap = (NOALLOC_SCRATCH_BYTES - head) / (10 * (int64_t)sizeof(double));
    if (cap < n_act)
        return NBODY_EINVAL;   // records plus one split of partials exceed the scratch
    if (hipGetDevice(&c.device) != hipSuccess)
        return NBODY_EDEVICE;
    unsigned char *base = nullptr;
    if (scratch_address(c.device, &base) != hipSuccess)
        return NBODY_EDEVICE;
    noalloc_layout(n, precision, &c, base, &seg, &off);
    c.part = reinterpret_cast<double *>(base + head);
    c.part_cap = cap;
    const Launch L = rule_launch(n_act, n, cap, precision);
    const int64_t ib = iblock_size(L);
    ForceWork w{};
    w.idx = d_idx;
    w.seg = seg;
    w.off = off;
    w.split = L.split;
    w.nc = 1;
    w.n_blocks = (n_act + ib - 1) / ib;
    ForceOut out{};
    out.vec[0] = d_acc_out;
    out.vec[1] = d_jrk_out;
    out.vec[2] = d_snp_out;
    out.pot = d_pot_out;
    out.sk = 3;
    out.sd = 1;
    if (launch_pack_arrays(c, d_mass, d_pos, d_vel, d_acc, n_act, seg, off, c.stream) !=
            hipSuccess ||
        launch_force(c, w, L, out, n_act, c.stream) != hipSuccess)
        return NBODY_EDEVICE;
    return NBODY_OK;
}

int64_t nbody_profile_force_log(nbody_ctx *ctx, int64_t max, int64_t *n_act, double *pairs,
                                double *ms)
{
    if (!ctx)
        return NBODY_EINVAL;
    Ctx &c = ctx->c;
    if (prof_collect(c) != hipSuccess)
        return NBODY_EDEVICE;
    const int64_t n = (int64_t)c.flog_ms.size();
    for (int64_t k = 0; k < std::min(n, max); ++k) {
        if (n_act)
            n_act[k] = c.flog_nact[k];
        if (pairs)
            pairs[k] = c.flog_pairs[k];
        if (ms)
            ms[k] = c.flog_ms[k];
    }
    return n;
}

}  // extern "C"
