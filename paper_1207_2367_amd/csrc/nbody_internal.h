// Internal declarations of the gfx950 N-body library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <string>
#include <vector>

#include "nbody.h"

namespace nb {

// ---------------------------------------------------------------- records
// Source ("j") records: the predicted state of every particle at the block
// time, structure-of-arrays so that a tile load is coalesced.
//   mixed    : x, y, z, mass and velocity in FP64 (they enter the FP64
//              acceleration, jerk and potential), acceleration in FP32
//              (it enters only the FP32 snap)          -> 68 bytes
//   FP32 pair: x, y, z and mass in FP64, velocity and acceleration in
//              FP32                                    -> 56 bytes
//   fp64     : every field FP64                        -> 80 bytes per particle
template <typename VT>
struct JRecMix {
    double *x, *y, *z, *m;
    VT *vx, *vy, *vz;
    float *ax, *ay, *az;
};
using JRecMixed = JRecMix<double>;
using JRecPair32 = JRecMix<float>;
struct JRecF64 {
    double *x, *y, *z, *vx, *vy, *vz, *ax, *ay, *az, *m;
    double *jx, *jy, *jz;   // sources' jerks: start-up evaluation only
};

// Hermite state, FP64 structure-of-arrays: component d of particle i of
// field f is f[d * n + i].  176 bytes per particle.
struct State {
    double *pos, *vel, *acc, *jrk, *snp, *crk;  // [3][n]
    double *t, *dt, *mass;                      // [n]
};

// Where a force evaluation writes: component d of output q (0 acc, 1 jrk,
// 2 snp, 3 crackle -- start-up evaluation only) of active slot k goes to
// vec[q][k * sk + d * sd]; the potential to pot[k].  A null vec[q] or pot
// is not written.
struct ForceOut {
    double *vec[4];
    double *pot;
    int64_t sk, sd;
};

// Work layout of one force launch over clusters.  Active slot k in
// [seg[c], seg[c+1]) belongs to cluster c whose sources are
// [off[c], off[c+1]).  i-block g of the launch covers slots
// [seg[c] + (g - blk_first[c]) * IB, ...) of cluster c = blk_cluster[g]
// (blk_cluster == nullptr: a single cluster, c = 0, blk_first = 0).
struct ForceWork {
    const int32_t *idx;       // active particle of each slot
    const int64_t *seg;       // [nc + 1] device
    const int64_t *off;       // [nc + 1] device
    const int32_t *blk_cluster;
    const int64_t *blk_first;
    int64_t n_blocks;         // i-blocks in the grid (x dimension)
    int32_t split;            // B, the split-source factor (grid y)
    int32_t nc;
    // error word for an active particle outside its cluster's sources (a
    // caller's bad index list; the slot is skipped), or nullptr
    uint32_t *err;
};

// Launch shape of the evaluation: lanes per active particle, waves per
// workgroup, split-source factor, active particles per lane group (1 or 2;
// 2 only with lpi <= 4).
// Work split of the ensemble loop (independent clusters in one persistent
// launch): group g holds the size[g] consecutive workgroups from first[g]
// and integrates the clusters cl[cl_off[g] .. cl_off[g+1]) one after
// another, with its split partials in slots [part_off[g], + part_cap[g]).
// Device arrays in the workspace.
struct EnsPlan {
    const int32_t *grp_of;     // [G] group of each workgroup
    const int32_t *first;      // [ng] first workgroup of the group
    const int32_t *size;       // [ng] workgroups of the group
    const int32_t *cl;         // [nc] clusters, group after group
    const int32_t *cl_off;     // [ng + 1]
    const int64_t *part_off;   // [ng]
    const int64_t *part_cap;   // [ng]
    int64_t *seg;              // [2 ng] active segment of the group's cluster
};

struct Launch {
    int lpi = 0, waves = 0, split = 0, ipt = 1;
};

// Sources per split of a cluster of nsrc sources under split factor B with
// tiles of nt: ceil(nsrc / B) rounded up to whole tiles; the splits in use
// are those that start below nsrc (at least one).
__host__ __device__ inline int64_t split_chunk(int64_t nsrc, int64_t B, int64_t nt)
{
    const int64_t c = (nsrc + B - 1) / B;
    return (c + nt - 1) / nt * nt;
}
__host__ __device__ inline int64_t splits_used(int64_t nsrc, int64_t B, int64_t nt)
{
    const int64_t c = split_chunk(nsrc, B, nt);
    const int64_t u = c > 0 ? (nsrc + c - 1) / c : 1;
    return u < 1 ? 1 : u;
}

struct Ctx;

// force.hip
hipError_t launch_force(Ctx &c, const ForceWork &w, const Launch &L,
                        const ForceOut &out, int64_t n_act_total, hipStream_t s,
                        bool reduce = true);
hipError_t launch_reduce_correct(const Ctx &c, const ForceWork &w, int split, int nt,
                                 int64_t n_act, double t_target, hipStream_t s,
                                 bool levels = false);
Launch pick_launch(const Ctx &c, int64_t n_act, int64_t n_src_max);
Launch rule_launch(int64_t n_act, int64_t n_src, int64_t part_cap, int prec);
// start-up evaluation (FP64, a, da, d2a and crackle of every particle from
// the stored state): split = 1, results written straight to out
hipError_t launch_energy_pot(Ctx &c, double *phi, hipStream_t s);
hipError_t launch_force_init(Ctx &c, const ForceWork &w, const Launch &L,
                             const ForceOut &out, hipStream_t s);
int64_t iblock_size(const Launch &L);

// integrate.hip
hipError_t launch_pack(const Ctx &c, const double *T_cluster, int own_time,
                       const int32_t *cluster_of, hipStream_t s);
// records of c.n particles from caller arrays (c.jm / c.jp / c.jd per the
// precision), plus seg = {0, n_act} and off = {0, c.n}
hipError_t launch_pack_arrays(const Ctx &c, const double *mass, const double *pos,
                              const double *vel, const double *acc, int64_t n_act,
                              int64_t *seg, int64_t *off, hipStream_t s);
hipError_t launch_predict_out(const Ctx &c, double t, double *pos, double *vel,
                              double *acc, hipStream_t s);
hipError_t launch_schedule(const Ctx &c, double t_target, int64_t seq, hipStream_t s);
hipError_t launch_sched_reset(const Ctx &c, hipStream_t s);
hipError_t launch_sched_head(const Ctx &c, double t_target, int64_t seq, hipStream_t s);
// per-level counts of the stored state, the time of the last block and the
// check that every step is a power of two within [dt_min, dt_max] and every
// particle's time a multiple of its step below the next one (d_lvl[LVL_BAD])
hipError_t launch_levels_build(const Ctx &c, hipStream_t s);
// the schedule of the next block from the counts (as launch_sched_head)
hipError_t launch_levels_sched(const Ctx &c, double t_target, int64_t seq, hipStream_t s);
hipError_t launch_sched_scatter(const Ctx &c, hipStream_t s);
// compaction of the active list and predictor; with levels, the active list
// is filled through an atomic position (chunks in any order)
hipError_t launch_scatter_pack(const Ctx &c, hipStream_t s, bool levels = false);
hipError_t launch_step_loop(const Ctx &c, double t_target, int64_t a_max, int grid, int64_t seq,
                            hipStream_t s);
// workgroups of the device-resident loop that can be resident at once for
// the context's precision (0 if the device cannot launch it cooperatively)
int step_loop_max_grid(const Ctx &c);
// the same for the ensemble loop (every resident workgroup, <= LOOP_GMAX)
int ensemble_max_grid(const Ctx &c);
hipError_t launch_ensemble_loop(const Ctx &c, double t_target, int grid, const EnsPlan &plan,
                                unsigned long long *res, hipStream_t s);
hipError_t launch_blocks(const Ctx &c, int64_t ib, int64_t cap, hipStream_t s);
hipError_t launch_segments(const Ctx &c, const int32_t *idx, int64_t n_act, hipStream_t s);
hipError_t launch_correct(const Ctx &c, int64_t n_act, const int32_t *idx,
                          double t_target, const double *fa, const double *fj,
                          const double *fs, int64_t sk, int64_t sd, hipStream_t s,
                          bool levels = false);
hipError_t launch_recap(const Ctx &c, double t_target, hipStream_t s);
hipError_t launch_energy_sums(const Ctx &c, const double *phi, double *out5,
                              hipStream_t s);
hipError_t launch_validate_idx(const Ctx &c, int64_t n_act, const int32_t *idx,
                               hipStream_t s);
// ERR_STATE unless every cluster's particles share one time
hipError_t launch_sync_check(const Ctx &c, hipStream_t s);
hipError_t launch_aos_to_soa(const double *src, double *dst, int64_t n,
                             hipStream_t s);
hipError_t launch_soa_to_aos(const double *src, double *dst, int64_t n,
                             hipStream_t s);
hipError_t launch_check_finite(const Ctx &c, hipStream_t s);
hipError_t launch_init_dt(const Ctx &c, hipStream_t s);

// Device error word bits (set with atomicOr by kernels).
enum : uint32_t {
    ERR_DTMIN = 1u, ERR_NONFINITE = 2u, ERR_BADIDX = 4u, ERR_LOOP = 8u, ERR_STATE = 16u,
    ERR_LEVELS = 32u
};

// Schedule from per-level counts (a single system, nbody_step): lvl[k] =
// number of particles whose step is dt_max 2^-k (k < LVL_N), then the time
// of the last block (as bits), a violation flag, the active list's fill
// position and the N_act the schedule announced.
constexpr int LVL_N = 64;
enum : int { LVL_TPREV = LVL_N, LVL_BAD = LVL_N + 1, LVL_POS = LVL_N + 2, LVL_NACT = LVL_N + 3,
             LVL_WORDS = LVL_N + 4 };

// Device-resident block-step loop: why it stopped, and the largest grid.
enum : int { LOOP_DONE = 1, LOOP_BIG = 2, LOOP_ERR = 3 };
constexpr int LOOP_GMAX = 1024;
constexpr int LOOP_GRID = 64;            // workgroups the loop uses
constexpr int64_t LOOP_AUTO_NMAX = 4096; // automatic mode: systems up to this size
constexpr int64_t LOOP_BAR_WORDS = 32 * LOOP_GMAX;         // barrier lines (128 B each)
// largest group of the ensemble loop (a barrier's cost grows with the
// group's size: beyond 256 workgroups it outweighs the extra lanes)
constexpr int ENS_GROUP_MAX = 256;

// Schedule scratch: chunk table built at init (a chunk never spans two
// clusters), per-cluster block times and active segments.
constexpr int SCHED_CHUNK = 2048;

// Event-based timing of the phases of a block step (host side).
enum Phase { PH_SCHED = 0, PH_PREDICT, PH_FORCE, PH_REDUCE, PH_CORRECT, PH_ENERGY, PH_N };
struct ProfRec {
    int phase;
    hipEvent_t a, b;
    int64_t n_act;
    double pairs;
};

struct Ctx {
    int64_t n = 0;
    int32_t nc = 1;
    double eps = 0.0;
    nbody_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    State st{};
    JRecMixed jm{};
    JRecPair32 jp{};
    JRecF64 jd{};
    // [nc + 1] device copies of the cluster offsets, host copy too
    int64_t *d_off = nullptr;
    std::vector<int64_t> off;
    int32_t *d_cluster_of = nullptr;  // [n] cluster of each particle (nc > 1)
    // split-source partials: [B][10][n_act]
    double *part = nullptr;
    int64_t part_cap = 0;              // capacity in (B * n_act) units
    // active list and new forces of the integrator: fnew[10][n]
    int32_t *act = nullptr;
    double *fnew = nullptr;
    // scheduling
    int64_t n_chunks = 0;
    int32_t *d_chunk_cluster = nullptr;  // [n_chunks]
    int64_t *d_chunk_begin = nullptr;    // [n_chunks + 1]
    uint64_t *d_tmin = nullptr;          // [nc] bits of min(t+dt), per cluster
    double *d_tblock = nullptr;          // [nc] block time, +inf if done
    int32_t *d_chunk_cnt = nullptr;      // [n_chunks] particles at the chunk's minimum
    uint64_t *d_chunk_min = nullptr;     // [n_chunks] chunk minimum of t + dt (bits)
    int64_t *d_chunk_pos = nullptr;      // [n_chunks]
    int64_t *d_seg = nullptr;            // [nc + 1] active segments
    int32_t *d_blk_cluster = nullptr;    // [n / 1 + nc] i-block -> cluster
    int64_t *d_blk_first = nullptr;      // [nc + 1]
    int64_t *d_info = nullptr;           // [64]: [0..7] step info, [8..47] N_act histogram
    uint32_t *d_err = nullptr;           // device error word
    double *d_red = nullptr;             // reduction scratch
    int64_t red_cap = 0;
    double *d_phi = nullptr;             // [n] potential scratch (energy)
    // host pinned mirror for small readbacks
    int64_t *h_info = nullptr;
    int64_t *h_tot = nullptr;            // [8] scheduler totals, written by the GPU (mapped):
                                         // [0..5] totals, [6] sequence number of the schedule
    int64_t sched_seq = 0;               // sequence number of the last schedule launched
    int64_t loop_seq = 0;                // same for the device-resident loop (h_tot[15])
    int64_t loop_amax = -1;              // loop's largest N_act: -1 automatic, 0 off
    int64_t *d_lvl = nullptr;            // [LVL_WORDS] per-level counts (see LVL_N)
    int sched_mode = 0;                  // 0: per-level counts where valid, 1: sweep only
    int loop_grid = -1;                  // its workgroups (-1: not yet queried, 0: none)
    uint64_t *d_loop_min = nullptr;      // [2 LOOP_GMAX] per-workgroup minima (two banks)
    int32_t *d_loop_cnt = nullptr;       // [2 LOOP_GMAX] and counts
    // ensemble loop: plan tables (device, in the workspace), its grid (-1
    // not yet planned, 0 unavailable), and its result counters
    EnsPlan ens{};
    int32_t *d_ens_i32 = nullptr;        // grp_of, first, size, cl_off, cl
    int64_t *d_ens_i64 = nullptr;        // part_off, part_cap, seg
    int ens_grid = -1;
    unsigned long long *d_ens_res = nullptr;   // [4]
    uint32_t *d_loop_bar = nullptr;      // [2 LOOP_BAR_WORDS] barrier words, then the ensemble
                                         // groups' unit counters (a line per group)
    int64_t *d_tot = nullptr;            // device address of h_tot
    double *h_red = nullptr;
    uint32_t *h_err = nullptr;
    // profiling
    bool prof = false;
    std::vector<ProfRec> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    double prof_ms[PH_N] = {0};
    int64_t prof_cnt[PH_N] = {0};
    double prof_pairs = 0.0;
    std::vector<int64_t> flog_nact;
    std::vector<double> flog_pairs, flog_ms;
    // launch choice
    Launch pinned{};
    std::vector<Launch> tuned;  // index: floor(log2(n_act))
    std::string last_error;
};

int64_t ws_layout(int64_t n, int32_t nc, int32_t prec, Ctx *c, char *base);

// profiling marks (no-ops unless c.prof); prof_begin returns a record index
int prof_begin(Ctx &c, int phase, int64_t n_act = 0, double pairs = 0.0);
void prof_end(Ctx &c, int rec);
hipError_t prof_collect(Ctx &c);

}  // namespace nb
