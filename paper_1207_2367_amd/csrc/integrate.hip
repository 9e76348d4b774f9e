// Block-time-step machinery of the Hermite scheme on gfx950: prediction of
// the sources (paper Sect. 3, item 1), active-set selection (Table 1,
// section 1), corrector (item 3), interpolation of the higher derivatives,
// the generalized Aarseth criterion (Eqs. indtstp, As) with power-of-two
// block rules, and the energy / angular-momentum sums (Sect. 5.1).
//
// These kernels stream O(N) or O(N_act) FP64 data once, so the bound is HBM
// bandwidth (or, for small sets, latency): they read structure-of-arrays
// state with one particle per lane (coalesced), keep every per-particle
// temporary in registers and write each output once.  Reductions run in a
// fixed tree order, so two identical runs give identical bits.  The file
// also holds the schedule from per-level counts of the power-of-two steps
// (levels_*), the device-resident loop that runs whole block steps of a
// small system inside one cooperative launch (step_loop_kernel) and the
// ensemble loop that runs every block step of every cluster of a batched
// context in one launch (ensemble_loop_kernel), both with the evaluation
// body of force_body.h.
#include <cfloat>
#include <cmath>

#include "force_body.h"

namespace nb {

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ double pow2_floor(double x)
{
    // largest power of two <= x for a positive normal x: keep the exponent
    return __longlong_as_double(__double_as_longlong(x) & (long long)0xFFF0000000000000ULL);
}

// Per-level counts (a schedule from levels): level of a power-of-two step,
// dt = 2^(e0 - k) with e0 the exponent of dt_max.
__device__ __forceinline__ int dt_level(double dt, int e0)
{
    return e0 - ((int)((__double_as_longlong(dt) >> 52) & 0x7FF) - 1023);
}

__device__ __forceinline__ double norm3(double x, double y, double z)
{
    return sqrt(x * x + y * y + z * z);
}

// Block rules (reading of the paper's power-of-two quantization): round the
// criterion down to a power of two, clamp to [dt_min, dt_max]; grow only by
// doubling and only where t_new is a multiple of 2 dt_old; shrink freely;
// while short of t_target, halve until t_new + dt <= t_target.
// Returns 0, ERR_DTMIN or ERR_NONFINITE.
__device__ uint32_t block_dt(double crit, double dt_old, double t_new, double t_target,
                             double dt_min, double dt_max, double *dt_out)
{
    if (crit != crit)
        return ERR_NONFINITE;
    if (crit < dt_min)
        return ERR_DTMIN;
    double dt = dt_max;
    if (crit < dt_max) {
        dt = pow2_floor(crit);
        if (dt < dt_min)
            dt = dt_min;
    }
    if (dt_old > 0.0 && dt > dt_old) {
        const double q = t_new / (2.0 * dt_old);   // exact: dyadic / power of two
        dt = (q == floor(q)) ? 2.0 * dt_old : dt_old;
    }
    if (t_new < t_target) {
        for (int it = 0; it < 80 && t_new + dt > t_target; ++it)
            dt *= 0.5;
    }
    if (dt < dt_min)
        return ERR_DTMIN;
    *dt_out = dt;
    return 0;
}

// ------------------------------------------------------------- predictor
// Taylor series of paper Sect. 3 item 1 (Horner form) to the source
// records.  T is the block time of the particle's cluster, or its own time
// (h = 0: the records are the stored state) when own_time is set.
__device__ __forceinline__ void pack_h(const State &st, const JRecMixed &jm,
                                       const JRecPair32 &jp, const JRecF64 &jd, int prec,
                                       int64_t n, int64_t i, double h);

__device__ __forceinline__ void pack_one(const State &st, const JRecMixed &jm,
                                         const JRecPair32 &jp, const JRecF64 &jd, int prec,
                                         int64_t n,
                                         const double *Tc, const int32_t *cluster_of,
                                         int own_time, int64_t i)
{
    if (i >= n)
        return;
    double h = 0.0;
    if (!own_time) {
        const double T = Tc[cluster_of ? cluster_of[i] : 0];
        if (!(T < DBL_MAX))
            return;  // cluster has reached the target: not a source this step
        h = T - st.t[i];
    }
    pack_h(st, jm, jp, jd, prec, n, i, h);
}

// the stored state of particle i that its prediction reads
struct PredIn {
    double x[3], v[3], a[3], j[3], s[3], c[3], m, t;
};

__device__ __forceinline__ PredIn load_pred(const State &st, int64_t n, int64_t i)
{
    PredIn q;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int64_t e = (int64_t)d * n + i;
        q.x[d] = st.pos[e];
        q.v[d] = st.vel[e];
        q.a[d] = st.acc[e];
        q.j[d] = st.jrk[e];
        q.s[d] = st.snp[e];
        q.c[d] = st.crk[e];
    }
    q.m = st.mass[i];
    q.t = st.t[i];
    return q;
}

__device__ __forceinline__ void store_pred(const PredIn &q, const JRecMixed &jm,
                                           const JRecPair32 &jp, const JRecF64 &jd, int prec,
                                           int64_t i, double h);

// the records of particle i advanced by h from its own time
__device__ __forceinline__ void pack_h(const State &st, const JRecMixed &jm,
                                       const JRecPair32 &jp, const JRecF64 &jd, int prec,
                                       int64_t n, int64_t i, double h)
{
    store_pred(load_pred(st, n, i), jm, jp, jd, prec, i, h);
}

// the records of the particles [r0, r1) of one workgroup advanced to T, two
// particles per lane and pass with all loads of both issued before either
// particle's stores (the stores could alias the loads as far as the
// compiler knows, so it would not overlap two passes by itself)
__device__ __forceinline__ void pack_range(const State &st, const JRecMixed &jm,
                                           const JRecPair32 &jp, const JRecF64 &jd, int prec,
                                           int64_t n, int64_t r0, int64_t r1, double T)
{
    for (int64_t i = r0 + threadIdx.x; i < r1; i += 2 * TPB) {
        const int64_t i2 = i + TPB;
        const bool two = i2 < r1;
        const PredIn a = load_pred(st, n, i);
        PredIn b{};
        if (two)
            b = load_pred(st, n, i2);
        store_pred(a, jm, jp, jd, prec, i, T - a.t);
        if (two)
            store_pred(b, jm, jp, jd, prec, i2, T - b.t);
    }
}

__device__ __forceinline__ void store_pred(const PredIn &q, const JRecMixed &jm,
                                           const JRecPair32 &jp, const JRecF64 &jd, int prec,
                                           int64_t i, double h)
{
    double xp[3], vp[3], ap[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double x = q.x[d], v = q.v[d], a = q.a[d];
        const double j = q.j[d], s = q.s[d], c = q.c[d];
        xp[d] = x + h * (v + h * (a * 0.5 + h * (j * (1.0 / 6) + h * (s * (1.0 / 24) + h * (c * (1.0 / 120))))));
        vp[d] = v + h * (a + h * (j * 0.5 + h * (s * (1.0 / 6) + h * (c * (1.0 / 24)))));
        ap[d] = a + h * (j + h * (s * 0.5 + h * (c * (1.0 / 6))));
    }
    const double m = q.m;
    if (prec == NBODY_PREC_MIXED) {
        jm.x[i] = xp[0]; jm.y[i] = xp[1]; jm.z[i] = xp[2];
        jm.vx[i] = vp[0]; jm.vy[i] = vp[1]; jm.vz[i] = vp[2];
        jm.ax[i] = (float)ap[0]; jm.ay[i] = (float)ap[1]; jm.az[i] = (float)ap[2];
        jm.m[i] = m;
    } else if (prec == NBODY_PREC_FP32PAIR) {
        jp.x[i] = xp[0]; jp.y[i] = xp[1]; jp.z[i] = xp[2];
        jp.vx[i] = (float)vp[0]; jp.vy[i] = (float)vp[1]; jp.vz[i] = (float)vp[2];
        jp.ax[i] = (float)ap[0]; jp.ay[i] = (float)ap[1]; jp.az[i] = (float)ap[2];
        jp.m[i] = m;
    } else {
        jd.x[i] = xp[0]; jd.y[i] = xp[1]; jd.z[i] = xp[2];
        jd.vx[i] = vp[0]; jd.vy[i] = vp[1]; jd.vz[i] = vp[2];
        jd.ax[i] = ap[0]; jd.ay[i] = ap[1]; jd.az[i] = ap[2];
        jd.m[i] = m;
    }
}

__global__ __launch_bounds__(TPB) void pack_kernel(State st, JRecMixed jm, JRecPair32 jp, JRecF64 jd,
                                                   int prec, int64_t n, const double *Tc,
                                                   const int32_t *cluster_of, int own_time)
{
    pack_one(st, jm, jp, jd, prec, n, Tc, cluster_of, own_time,
             (int64_t)blockIdx.x * TPB + threadIdx.x);
}

// Predictor to FP64 [n][3] outputs at a common time t (diagnostic entry).
__global__ __launch_bounds__(TPB) void predict_out_kernel(State st, int64_t n, double t,
                                                          double *po, double *vo, double *ao)
{
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n)
        return;
    const double h = t - st.t[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int64_t e = (int64_t)d * n + i;
        const double x = st.pos[e], v = st.vel[e], a = st.acc[e];
        const double j = st.jrk[e], s = st.snp[e], c = st.crk[e];
        po[3 * i + d] = x + h * (v + h * (a * 0.5 + h * (j * (1.0 / 6) + h * (s * (1.0 / 24) + h * (c * (1.0 / 120))))));
        vo[3 * i + d] = v + h * (a + h * (j * 0.5 + h * (s * (1.0 / 6) + h * (c * (1.0 / 24)))));
        ao[3 * i + d] = a + h * (j + h * (s * 0.5 + h * (c * (1.0 / 6))));
    }
}

// ---------------------------------------------------------- scheduling
__global__ void sched_reset(uint64_t *tmin, int32_t nc)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nc)
        tmin[c] = ~0ull;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint64_t o = __shfl_xor(v, m, 64);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint64_t o = __shfl_xor(v, m, 64);
        v = o > v ? o : v;
    }
    return v;
}

// per chunk: the minimum over its particles of t + dt (as ordered bits;
// times are >= 0 so the IEEE bits order like the values) and how many of
// its particles reach it; the minimum also goes into the cluster's slot.
// A chunk's particles are due exactly when its minimum is the cluster's.
__device__ __forceinline__ void min_count(uint64_t &v, int &n, uint64_t ov, int on)
{
    if (ov < v) {
        v = ov;
        n = on;
    } else if (ov == v) {
        n += on;
    }
}

__global__ __launch_bounds__(TPB) void sched_min(const double *t, const double *dt,
                                                 const int64_t *chunk_begin,
                                                 const int32_t *chunk_cluster, uint64_t *tmin,
                                                 uint64_t *cmin, int32_t *ccnt)
{
    __shared__ uint64_t rv[TPB / 64];
    __shared__ int rn[TPB / 64];
    const int64_t b = chunk_begin[blockIdx.x], e = chunk_begin[blockIdx.x + 1];
    uint64_t v = ~0ull;
    int n = 0;
    for (int64_t i = b + threadIdx.x; i < e; i += TPB)
        min_count(v, n, (uint64_t)__double_as_longlong(t[i] + dt[i]), 1);
    // xor butterfly: both partners form the same (min, count) of their union
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint64_t ov = __shfl_xor(v, m, 64);
        const int on = __shfl_xor(n, m, 64);
        min_count(v, n, ov, on);
    }
    if ((threadIdx.x & 63) == 0) {
        rv[threadIdx.x >> 6] = v;
        rn[threadIdx.x >> 6] = n;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < TPB / 64; ++w)
            min_count(v, n, rv[w], rn[w]);
        cmin[blockIdx.x] = v;
        ccnt[blockIdx.x] = n;
        atomicMin((unsigned long long *)&tmin[chunk_cluster[blockIdx.x]], (unsigned long long)v);
    }
}

__device__ __forceinline__ bool due(double t, double dt, double T) { return t + dt == T; }

// Single workgroup: the due count of every chunk (its count at its minimum
// when that is its cluster's block time and the cluster is not past the
// target), their exclusive scan (chunks are in particle order, so clusters
// are contiguous), per-cluster active segments and block times, totals and
// the N_act histogram.
// info[0] = N_act total, info[1] = bits of the earliest block time,
// info[2] = sum_c N_c * n_act,c, info[3] = device error word snapshot,
// info[4] = clusters with active particles, info[5] = the largest of them.
__device__ __forceinline__ void sched_scan_body(const uint64_t *cmin, const int32_t *ccnt,
                                                int64_t n_chunks, const int32_t *chunk_cluster,
                                                uint64_t *tmin, const int64_t *off, int32_t nc,
                                                double t_target, int64_t *chunk_pos,
                                                int64_t *seg, double *tblock, int64_t *info,
                                                int64_t *hist, const uint32_t *err,
                                                int64_t *info_host, int64_t seq)
{
    // exclusive scan of the due counts, 1024 chunks at a time: inclusive
    // scan inside each wave by shuffles, then the 16 wave totals
    __shared__ int64_t wtot[1024 / 64];
    __shared__ int64_t carry;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0)
        carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < n_chunks; base += 1024) {
        const int64_t q = base + threadIdx.x;
        int64_t v = 0;
        if (q < n_chunks) {
            // one system: every chunk belongs to cluster 0 (no dependent load)
            const uint64_t T = tmin[nc == 1 ? 0 : chunk_cluster[q]];
            if (cmin[q] == T && __longlong_as_double((long long)T) <= t_target)
                v = ccnt[q];
        }
        int64_t x = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t y = __shfl_up(x, d, 64);
            x += lane >= d ? y : 0;
        }
        if (lane == 63)
            wtot[wave] = x;
        __syncthreads();
        int64_t woff = 0, all = 0;
        for (int w = 0; w < 1024 / 64; ++w) {
            const int64_t t = wtot[w];
            woff += w < wave ? t : 0;
            all += t;
        }
        if (q < n_chunks)
            chunk_pos[q] = carry + woff + x - v;
        __syncthreads();
        if (threadIdx.x == 0)
            carry += all;
        __syncthreads();
    }
    // segment starts: position of the first chunk of each cluster
    if (nc == 1) {
        if (threadIdx.x == 0)
            seg[0] = 0;
    } else {
        for (int64_t q = threadIdx.x; q < n_chunks; q += 1024) {
            const int32_t c = chunk_cluster[q];
            if (q == 0 || chunk_cluster[q - 1] != c)
                seg[c] = chunk_pos[q];
        }
    }
    if (threadIdx.x == 0) {
        seg[nc] = carry;
        info[0] = carry;
    }
    __syncthreads();
    // per cluster (spread over the threads): block time, interactions and
    // the histogram; then the earliest time and the pair total
    __shared__ double rmin[1024 / 64];
    __shared__ int64_t rsum[1024 / 64], rcnt[1024 / 64], rbig[1024 / 64];
    double tmn = INFINITY;
    int64_t pairs = 0, nclus = 0, big = 0;
    for (int32_t c = threadIdx.x; c < nc; c += 1024) {
        const double T = __longlong_as_double((long long)tmin[c]);
        const bool act = T <= t_target;
        tblock[c] = act ? T : INFINITY;
        if (act && T < tmn)
            tmn = T;
        const int64_t na = seg[c + 1] - seg[c];
        const int64_t nsrc = off[c + 1] - off[c];
        pairs += na * nsrc;
        if (na > 0) {
            ++nclus;
            big = nsrc > big ? nsrc : big;
            int bb = 0;
            while ((int64_t(1) << (bb + 1)) <= na)
                ++bb;
            atomicAdd((unsigned long long *)&hist[bb], 1ull);
        }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const double o = __shfl_xor(tmn, m, 64);
        tmn = o < tmn ? o : tmn;
        pairs += __shfl_xor(pairs, m, 64);
        nclus += __shfl_xor(nclus, m, 64);
        const int64_t ob = __shfl_xor(big, m, 64);
        big = ob > big ? ob : big;
    }
    if ((threadIdx.x & 63) == 0) {
        rmin[threadIdx.x >> 6] = tmn;
        rsum[threadIdx.x >> 6] = pairs;
        rcnt[threadIdx.x >> 6] = nclus;
        rbig[threadIdx.x >> 6] = big;
    }
    __syncthreads();
    // every read of the per-cluster minima is done: leave them reset for the
    // next schedule (so that no separate reset launch is needed)
    for (int32_t c = threadIdx.x; c < nc; c += 1024)
        tmin[c] = ~0ull;
    if (threadIdx.x == 0) {
        for (int w = 1; w < 1024 / 64; ++w) {
            tmn = rmin[w] < tmn ? rmin[w] : tmn;
            pairs += rsum[w];
            nclus += rcnt[w];
            big = rbig[w] > big ? rbig[w] : big;
        }
        info[1] = __double_as_longlong(tmn);
        info[2] = pairs;
        info[3] = (int64_t)*err;
        info[4] = nclus;
        info[5] = big;
        if (info_host) {
            // the same totals straight into host memory (mapped, coherent),
            // then the schedule's sequence number with system-scope release
            // order: the host polls that word and reads the totals after it
            info_host[0] = carry;
            info_host[1] = __double_as_longlong(tmn);
            info_host[2] = pairs;
            info_host[3] = (int64_t)*err;
            info_host[4] = nclus;
            info_host[5] = big;
            __hip_atomic_store(&info_host[6], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

__global__ __launch_bounds__(1024) void sched_scan(const uint64_t *cmin, const int32_t *ccnt,
                                                   int64_t n_chunks, const int32_t *chunk_cluster,
                                                   uint64_t *tmin, const int64_t *off, int32_t nc,
                                                   double t_target, int64_t *chunk_pos,
                                                   int64_t *seg, double *tblock, int64_t *info,
                                                   int64_t *hist, const uint32_t *err,
                                                   int64_t *info_host, int64_t seq)
{
    sched_scan_body(cmin, ccnt, n_chunks, chunk_cluster, tmin, off, nc, t_target, chunk_pos, seg,
                    tblock, info, hist, err, info_host, seq);
}

// ordered compaction of the due particles of each chunk
__device__ __forceinline__ void scatter_range(const double *t, const double *dt, double T,
                                              int64_t b, int64_t e, int64_t pos, int32_t *act);

__device__ __forceinline__ void scatter_chunk(const double *t, const double *dt,
                                              const int64_t *chunk_begin,
                                              const int32_t *chunk_cluster,
                                              const double *tblock, const int64_t *chunk_pos,
                                              int32_t *act, int64_t q)
{
    const double T = tblock[chunk_cluster[q]];
    if (!(T < DBL_MAX))
        return;
    scatter_range(t, dt, T, chunk_begin[q], chunk_begin[q + 1], chunk_pos[q], act);
}

// the due particles of [b, e) in ascending order to act[pos ...]
__device__ __forceinline__ void scatter_range(const double *t, const double *dt, double T,
                                              int64_t b, int64_t e, int64_t pos, int32_t *act)
{
    __shared__ int wsum[TPB / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t base = b; base < e; base += TPB) {
        const int64_t i = base + threadIdx.x;
        const bool f = i < e && due(t[i], dt[i], T);
        const uint64_t mask = __ballot(f);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0)
            wsum[wave] = __popcll(mask);
        __syncthreads();
        int woff = 0, tot = 0;
        for (int w = 0; w < TPB / 64; ++w) {
            woff += w < wave ? wsum[w] : 0;
            tot += wsum[w];
        }
        if (f)
            act[pos + woff + before] = (int32_t)i;
        pos += tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(TPB) void sched_scatter(const double *t, const double *dt,
                                                     const int64_t *chunk_begin,
                                                     const int32_t *chunk_cluster,
                                                     const double *tblock,
                                                     const int64_t *chunk_pos, int32_t *act)
{
    scatter_chunk(t, dt, chunk_begin, chunk_cluster, tblock, chunk_pos, act, blockIdx.x);
}

// A block step's compaction and predictor in one launch: the first n_chunks
// workgroups compact one chunk each, the rest predict TPB sources each to
// their cluster's block time.  Both read only the schedule's results and
// the stored state; they write disjoint arrays.
// With fill != nullptr (one system, schedule from levels) a chunk counts its
// due particles, takes their place in the list with one atomic add on *fill
// and writes them in ascending order there (chunks land in any order; the
// evaluation and the corrector of a particle do not depend on its slot).
__device__ __forceinline__ void scatter_chunk_fill(const double *t, const double *dt, double T,
                                                   int64_t b, int64_t e, int32_t *act,
                                                   int64_t *fill)
{
    __shared__ int wcnt[TPB / 64];
    __shared__ int64_t base;
    int mine = 0;
    for (int64_t i = b + threadIdx.x; i < e; i += TPB)
        mine += due(t[i], dt[i], T) ? 1 : 0;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        mine += __shfl_xor(mine, m, 64);
    if ((threadIdx.x & 63) == 0)
        wcnt[threadIdx.x >> 6] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < TPB / 64; ++w)
            tot += wcnt[w];
        base = tot > 0 ? (int64_t)atomicAdd((unsigned long long *)fill, (unsigned long long)tot)
                       : 0;
    }
    __syncthreads();
    if (wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3] > 0)
        scatter_range(t, dt, T, b, e, base, act);
}

__global__ __launch_bounds__(TPB) void scatter_pack_kernel(State st, JRecMixed jm, JRecPair32 jp, JRecF64 jd,
                                                           int prec, int64_t n,
                                                           const int32_t *cluster_of,
                                                           const int64_t *chunk_begin,
                                                           const int32_t *chunk_cluster,
                                                           const double *tblock,
                                                           const int64_t *chunk_pos,
                                                           int32_t *act, int64_t n_chunks,
                                                           int64_t *fill)
{
    if ((int64_t)blockIdx.x < n_chunks && fill) {
        const double T = tblock[0];
        if (T < DBL_MAX)
            scatter_chunk_fill(st.t, st.dt, T, chunk_begin[blockIdx.x],
                               chunk_begin[blockIdx.x + 1], act, fill);
    } else if ((int64_t)blockIdx.x < n_chunks)
        scatter_chunk(st.t, st.dt, chunk_begin, chunk_cluster, tblock, chunk_pos, act,
                      blockIdx.x);
    else
        pack_one(st, jm, jp, jd, prec, n, tblock, cluster_of, 0,
                 ((int64_t)blockIdx.x - n_chunks) * TPB + threadIdx.x);
}

// ------------------------------------------ schedule from per-level counts
// For one system whose steps are powers of two dt_max 2^-k and whose
// particles each sit at a multiple of their step, below the next one
// (t_i <= T_last < t_i + dt_i, T_last the time of the last block), the next
// block time is the earliest next multiple of an occupied level's step after
// T_last, and the particles due then are exactly those of the levels whose
// step divides it; no sweep over the particles is needed.  The counts are
// built once per nbody_step call (and checked: any particle that breaks the
// conditions sets lvl[LVL_BAD], and the sweep is used instead) and kept up to
// date by the corrector.
__global__ __launch_bounds__(TPB) void levels_build_kernel(const double *t, const double *dt,
                                                           int64_t n, int e0, int kmax,
                                                           int64_t *lvl)
{
    __shared__ int cnt[LVL_N];
    if (threadIdx.x < LVL_N)
        cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    uint64_t tb = 0;
    if (i < n) {
        const double ti = t[i], di = dt[i];
        const uint64_t bits = (uint64_t)__double_as_longlong(di);
        const int k = dt_level(di, e0);
        // a power of two (zero mantissa, normal), on a level of [0, kmax],
        // a time that is a non-negative multiple of the step
        const bool ok = (bits & 0x000FFFFFFFFFFFFFull) == 0 && ((bits >> 52) & 0x7FF) != 0 &&
                        (bits >> 63) == 0 && k >= 0 && k <= kmax && k < LVL_N && ti >= 0.0 &&
                        floor(ti / di) * di == ti;
        if (ok)
            atomicAdd(&cnt[k], 1);
        else
            atomicOr((unsigned long long *)&lvl[LVL_BAD], 1ull);
        tb = ti >= 0.0 ? (uint64_t)__double_as_longlong(ti) : 0;
    }
    const uint64_t tm = wave_max_u64(tb);
    if ((threadIdx.x & 63) == 0)
        atomicMax((unsigned long long *)&lvl[LVL_TPREV], (unsigned long long)tm);
    __syncthreads();
    if (threadIdx.x < LVL_N && cnt[threadIdx.x] != 0)
        atomicAdd((unsigned long long *)&lvl[threadIdx.x], (unsigned long long)cnt[threadIdx.x]);
}

// second pass: every particle's next time lies beyond the last block
__global__ __launch_bounds__(TPB) void levels_check_kernel(const double *t, const double *dt,
                                                           int64_t n, int64_t *lvl)
{
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n)
        return;
    const double T = __longlong_as_double((long long)lvl[LVL_TPREV]);
    if (!(t[i] + dt[i] > T))
        atomicOr((unsigned long long *)&lvl[LVL_BAD], 1ull);
}

// One wave: the next block from the counts (the totals as sched_scan writes
// them, into info and the mapped host words with the sequence number), the
// time of the last block moved to it, and the active list's fill position
// cleared.  A fill position that does not match the N_act announced by the
// previous schedule (the compaction found other particles due than the counts
// said) sets ERR_LEVELS.
__global__ __launch_bounds__(64) void levels_sched_kernel(int64_t *lvl, int64_t n, int e0,
                                                          double t_target, int64_t *seg,
                                                          double *tblock, int64_t *info,
                                                          int64_t *hist, uint32_t *err,
                                                          int64_t *info_host, int64_t seq)
{
    const int k = threadIdx.x;
    const int64_t c = lvl[k];
    const double Tl = __longlong_as_double((long long)lvl[LVL_TPREV]);
    const double step = ldexp(1.0, e0 - k);
    const double next = c > 0 ? (floor(Tl / step) + 1.0) * step : INFINITY;
    double T = next;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const double o = __shfl_xor(T, m, 64);
        T = o < T ? o : T;
    }
    const bool act = T <= t_target;
    int64_t na = act && c > 0 && next == T ? c : 0;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        na += __shfl_xor(na, m, 64);
    if (k != 0)
        return;
    if (lvl[LVL_POS] != lvl[LVL_NACT])
        atomicOr(err, ERR_LEVELS);
    lvl[LVL_POS] = 0;
    lvl[LVL_NACT] = na;
    const double Tb = act ? T : INFINITY;
    if (na > 0) {
        lvl[LVL_TPREV] = __double_as_longlong(T);
        int bb = 0;
        while ((int64_t(1) << (bb + 1)) <= na)
            ++bb;
        atomicAdd((unsigned long long *)&hist[bb], 1ull);
    }
    seg[0] = 0;
    seg[1] = na;
    tblock[0] = na > 0 ? T : INFINITY;
    const int64_t tot[6] = {na, (int64_t)__double_as_longlong(Tb), na * n, (int64_t)*err,
                            na > 0 ? 1 : 0, n};
    for (int q = 0; q < 6; ++q) {
        info[q] = tot[q];
        info_host[q] = tot[q];
    }
    __hip_atomic_store(&info_host[6], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// i-block tables of a force launch over clusters: cluster c gets
// ceil(n_c / ib) blocks starting at blk_first[c] (an exclusive scan over the
// clusters, 1024 at a time, as in the schedule's scan); every grid slot g
// below the total then finds its cluster by a binary search over the starts
// (kept in LDS for up to BLK_LDS clusters), the rest of the grid (up to cap)
// is marked -1 (idle).  All of it in parallel: no loop over the clusters or
// over one cluster's blocks runs on a single lane.
constexpr int BLK_LDS = 8192;
__global__ __launch_bounds__(1024) void blocks_kernel(const int64_t *seg, int32_t nc, int64_t ib,
                                                      int64_t cap, int64_t *blk_first,
                                                      int32_t *blk_cluster)
{
    __shared__ int64_t buf[1024];
    __shared__ int32_t first[BLK_LDS];
    __shared__ int64_t carry;
    const bool in_lds = nc <= BLK_LDS;
    if (threadIdx.x == 0)
        carry = 0;
    __syncthreads();
    for (int32_t base = 0; base < nc; base += 1024) {
        const int32_t c = base + (int32_t)threadIdx.x;
        const int64_t v = c < nc ? (seg[c + 1] - seg[c] + ib - 1) / ib : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int s = 1; s < 1024; s <<= 1) {
            const int64_t add = threadIdx.x >= (unsigned)s ? buf[threadIdx.x - s] : 0;
            __syncthreads();
            buf[threadIdx.x] += add;
            __syncthreads();
        }
        if (c < nc) {
            const int64_t f = carry + buf[threadIdx.x] - v;
            blk_first[c] = f;
            if (in_lds)
                first[c] = (int32_t)f;
        }
        __syncthreads();
        if (threadIdx.x == 1023)
            carry += buf[1023];
        __syncthreads();
    }
    const int64_t total = carry;
    if (threadIdx.x == 0)
        blk_first[nc] = total;
    __syncthreads();
    for (int64_t g = threadIdx.x; g < cap; g += 1024) {
        int32_t cl = -1;
        if (g < total) {
            // the last cluster that starts at or before g (a cluster without
            // blocks starts where the next one does, so the last is the owner)
            int32_t lo = 0, hi = nc - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                const int64_t fm = in_lds ? (int64_t)first[mid] : blk_first[mid];
                if (fm <= g)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            cl = lo;
        }
        blk_cluster[g] = cl;
    }
}

// active segments of a caller's ascending index list: seg[c] = first slot
// whose particle is >= off[c]
__global__ void segments_kernel(const int32_t *idx, int64_t n_act, const int64_t *off,
                                int32_t nc, int64_t *seg)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nc)
        return;
    if (!idx) {  // identity list: every particle active
        seg[c] = off[c];
        return;
    }
    const int64_t key = off[c];
    int64_t lo = 0, hi = n_act;
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if ((int64_t)idx[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    seg[c] = c == nc ? n_act : lo;
}

__global__ void set_seg_kernel(int64_t *seg, int64_t a, int64_t b)
{
    seg[0] = a;
    seg[1] = b;
}

// ----------------------------------------------------------- corrector
// Corrector of paper Sect. 3 item 3 (velocity first, then position with the
// corrected velocity), end-of-step crackle/pop/5th derivative from the
// quintic through (a, da, d2a) at both ends, Aarseth criterion with p = 6,
// block rules.  h is the particle's own step; its block time is t + dt.
// Corrector (paper Sect. 3, item 3), interpolation of crackle, pop and the
// fifth derivative at the end of the step, and the new block step, for
// particle i with new a1, j1, s1 evaluated at t_i + dt_i.
// The stored state of particle i that the corrector reads (loaded apart
// from the arithmetic so that a kernel can issue these loads early).
struct OldState {
    double h, t, a0[3], j0[3], s0[3], v0[3], r0[3];
};

__device__ __forceinline__ OldState load_old(const State &st, int64_t n, int64_t i)
{
    OldState o;
    o.h = st.dt[i];
    o.t = st.t[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int64_t e = (int64_t)d * n + i;
        o.a0[d] = st.acc[e];
        o.j0[d] = st.jrk[e];
        o.s0[d] = st.snp[e];
        o.v0[d] = st.vel[e];
        o.r0[d] = st.pos[e];
    }
    return o;
}

__device__ __forceinline__ void correct_loaded(State st, int64_t n, int64_t i, const OldState &o,
                                               const double *a1, const double *j1,
                                               const double *s1, double t_target, double eta,
                                               double dt_min, double dt_max, uint32_t *err)
{
    const double h = o.h;
    const double t_new = o.t + h;
    double crk[3], pop[3], a5[3];
    uint32_t bad = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int64_t e = (int64_t)d * n + i;
        const double a0 = o.a0[d], j0 = o.j0[d], s0 = o.s0[d];
        const double v0 = o.v0[d], r0 = o.r0[d];
        const double v1 = v0 + h * 0.5 * (a1[d] + a0) - h * h * 0.1 * (j1[d] - j0) +
                          h * h * h * (1.0 / 120) * (s1[d] + s0);
        const double r1 = r0 + h * 0.5 * (v1 + v0) - h * h * 0.1 * (a1[d] - a0) +
                          h * h * h * (1.0 / 120) * (j1[d] + j0);
        // interpolation: C = c h^3, P = p h^4, X = x h^5 of the quintic
        const double D0 = a1[d] - a0 - h * j0 - 0.5 * h * h * s0;
        const double D1 = j1[d] - j0 - h * s0;
        const double D2 = s1[d] - s0;
        const double C = 60.0 * D0 - 24.0 * h * D1 + 3.0 * h * h * D2;
        const double P = -360.0 * D0 + 168.0 * h * D1 - 24.0 * h * h * D2;
        const double X = 720.0 * D0 - 360.0 * h * D1 + 60.0 * h * h * D2;
        const double ih = 1.0 / h;
        const double c0 = C * ih * ih * ih, p0 = P * ih * ih * ih * ih, x0 = X * ih * ih * ih * ih * ih;
        crk[d] = c0 + h * p0 + 0.5 * h * h * x0;
        pop[d] = p0 + h * x0;
        a5[d] = x0;
        if (!isfinite(r1) || !isfinite(v1))
            bad |= ERR_NONFINITE;
        st.pos[e] = r1;
        st.vel[e] = v1;
        st.acc[e] = a1[d];
        st.jrk[e] = j1[d];
        st.snp[e] = s1[d];
        st.crk[e] = crk[d];
    }
    const double A1 = sqrt(norm3(a1[0], a1[1], a1[2]) * norm3(s1[0], s1[1], s1[2]) +
                           j1[0] * j1[0] + j1[1] * j1[1] + j1[2] * j1[2]);
    const double A4 = sqrt(norm3(crk[0], crk[1], crk[2]) * norm3(a5[0], a5[1], a5[2]) +
                           pop[0] * pop[0] + pop[1] * pop[1] + pop[2] * pop[2]);
    const double crit = A4 == 0.0 ? INFINITY : eta * cbrt(A1 / A4);
    double dtn = h;
    bad |= block_dt(crit, h, t_new, t_target, dt_min, dt_max, &dtn);
    st.t[i] = t_new;
    if (!bad)
        st.dt[i] = dtn;
    if (bad)
        atomicOr(err, bad);
}

__device__ __forceinline__ void correct_one(State st, int64_t n, int64_t i, const double *a1,
                                            const double *j1, const double *s1,
                                            double t_target, double eta, double dt_min,
                                            double dt_max, uint32_t *err)
{
    correct_loaded(st, n, i, load_old(st, n, i), a1, j1, s1, t_target, eta, dt_min, dt_max, err);
}

// a workgroup's changes of the per-level counts (old step -> new step of the
// particles it corrected), gathered in LDS and added to lvl[] once per level
struct LevelDelta {
    int *d;
    __device__ void init()
    {
        __shared__ int sd[LVL_N];
        d = sd;
        if (threadIdx.x < LVL_N)
            d[threadIdx.x] = 0;
    }
    __device__ void move(double dt_old, double dt_new, int e0)
    {
        const int a = dt_level(dt_old, e0), b = dt_level(dt_new, e0);
        if (a != b && a >= 0 && a < LVL_N && b >= 0 && b < LVL_N) {
            atomicAdd(&d[a], -1);
            atomicAdd(&d[b], 1);
        }
    }
    __device__ void flush(int64_t *lvl)
    {
        if (threadIdx.x < LVL_N && d[threadIdx.x] != 0)
            atomicAdd((unsigned long long *)&lvl[threadIdx.x],
                      (unsigned long long)(int64_t)d[threadIdx.x]);
    }
};

// lvl: per-level counts to keep up to date (nullptr: none), e0 the exponent
// of dt_max
__global__ __launch_bounds__(TPB) void correct_kernel(
    State st, int64_t n, int64_t n_act, const int32_t *idx, double t_target,
    const double *fa, const double *fj, const double *fs, int64_t sk, int64_t sd,
    double eta, double dt_min, double dt_max, uint32_t *err, int64_t *lvl, int e0)
{
    LevelDelta ld;
    if (lvl) {
        ld.init();
        __syncthreads();
    }
    const int64_t k = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (k < n_act) {
        const int32_t i = idx[k];
        if (i < 0 || i >= n) {   // a caller's list out of range: report, touch nothing
            atomicOr(err, ERR_BADIDX);
        } else {
            double a1[3], j1[3], s1[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                a1[d] = fa[k * sk + d * sd];
                j1[d] = fj[k * sk + d * sd];
                s1[d] = fs[k * sk + d * sd];
            }
            const OldState o = load_old(st, n, i);
            correct_loaded(st, n, i, o, a1, j1, s1, t_target, eta, dt_min, dt_max, err);
            if (lvl)
                ld.move(o.h, st.dt[i], e0);
        }
    }
    if (lvl) {
        __syncthreads();
        ld.flush(lvl);
    }
}

// Split-source reduction and corrector of a block step in one kernel: a
// workgroup takes S active slots; R threads per (q, slot) sum quantity q
// (a, da, d2a components) over the splits that hold the slot's cluster, in
// a fixed order with 16 loads in flight, into LDS; then one thread per slot
// runs the corrector on the sums.  part is the evaluation's [B][10][n_act]
// buffer (the potential slot is not used).  The loops' own corrector phases
// take RC_SLOTS slots with one thread per sum.
constexpr int RC_SLOTS = TPB / 9;

// sum of bc split partials p[0], p[stride], ... in the order b = 0 .. bc-1,
// 16 loads in flight
__device__ __forceinline__ double sum_splits(const double *p, int64_t stride, int64_t bc)
{
    constexpr int U = 16;
    double r = 0.0;
    int64_t b = 0;
    for (; b + U <= bc; b += U) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            v[u] = p[(b + u) * stride];
#pragma unroll
        for (int u = 0; u < U; ++u)
            r += v[u];
    }
    for (; b < bc; ++b)
        r += p[b * stride];
    return r;
}

// R lanes per (quantity, slot): lane r sums the splits [r bc / R, (r + 1)
// bc / R) in order, and the corrector adds the R sums in the order r = 0 ..
// R-1 (R = 1: one lane sums all splits in order).  More lanes per sum cut
// the chain of dependent loads when a small block has many splits.
template <int R>
__global__ __launch_bounds__(TPB) void reduce_correct_kernel(
    State st, int64_t n, int64_t n_act, const double *part, int32_t B, int nt, ForceWork w,
    const int32_t *cluster_of, double t_target, double eta, double dt_min, double dt_max,
    uint32_t *err, int64_t *lvl, int e0)
{
    constexpr int S = TPB / (9 * R);   // active slots per workgroup
    __shared__ double ps[9][S][R];
    LevelDelta ld;
    if (lvl)
        ld.init();
    const int t = threadIdx.x;
    const int64_t k0 = (int64_t)blockIdx.x * S;
    // corrector lanes: t < S takes slot t.  An index outside the system (an
    // active list that does not match the schedule) is reported and the slot
    // left alone.
    const int64_t kc = k0 + t;
    const int64_t ic = t < S && kc < n_act ? w.idx[kc] : -1;
    if (t < S && kc < n_act && !(ic >= 0 && ic < n))
        atomicOr(err, ERR_BADIDX);
    const bool corr = ic >= 0 && ic < n;
    // summing lanes: (quantity q, slot kl, part r)
    const int qk = t / R, r = t % R, q = qk / S, kl = qk % S;
    const int64_t ks = k0 + kl;
    const int64_t is = q < 9 && ks < n_act ? w.idx[ks] : -1;
    // the lanes that run the corrector load its old state first, so that
    // those loads overlap the partial sums
    OldState o{};
    if (corr)
        o = load_old(st, n, ic);
    if (is >= 0 && is < n) {
        const int c = cluster_of ? cluster_of[is] : 0;
        const int64_t bc = splits_used(w.off[c + 1] - w.off[c], B, nt);
        const int64_t b0 = r * bc / R, b1 = (r + 1) * bc / R;
        ps[q][kl][r] = sum_splits(part + (int64_t)q * n_act + ks + b0 * 10 * n_act, 10 * n_act,
                                  b1 - b0);
    }
    __syncthreads();
    if (corr) {
        double f[9];
#pragma unroll
        for (int qq = 0; qq < 9; ++qq) {
            double v = ps[qq][t][0];
#pragma unroll
            for (int rr = 1; rr < R; ++rr)
                v += ps[qq][t][rr];
            f[qq] = v;
        }
        const double a1[3] = {f[0], f[1], f[2]};
        const double j1[3] = {f[3], f[4], f[5]};
        const double s1[3] = {f[6], f[7], f[8]};
        correct_loaded(st, n, ic, o, a1, j1, s1, t_target, eta, dt_min, dt_max, err);
        if (lvl)
            ld.move(o.h, st.dt[ic], e0);
    }
    if (lvl) {
        __syncthreads();
        ld.flush(lvl);
    }
}

// ------------------------------------------- device-resident block steps
// Block steps of one system whose active sets stay small, run inside one
// cooperative launch of G workgroups of TPB lanes (all resident at once),
// with three grid barriers per step:
//   (1) each workgroup sweeps its own particle range [r0, r1) for the
//       minimum of t + dt and how many particles reach it -> barrier;
//   (2) every workgroup reads the G results and forms the block time T,
//       N_act and the offset of its own due particles (the same decisions
//       everywhere); all stop together when nothing is due up to the target,
//       when N_act exceeds a_max (the host path takes that block) or when
//       the error word is set; otherwise each writes the ascending active
//       list of its range and predicts its range's sources to T -> barrier;
//   (3) the evaluation units (i-blocks of active particles against one of
//       B source splits, shaped as in the ensemble loop) are taken from a
//       shared counter -> barrier;
//   (4) each workgroup sums the split partials of its own range's active
//       particles in the order b = 0 .. B-1 and runs the corrector on them.
// The next sweep (1) reads only the workgroup's own range, which only that
// workgroup has changed in (4): a workgroup barrier is enough there.
constexpr int LOOP_NW = 4;                                // waves per workgroup
constexpr int LOOP_NT = LOOP_NW * 64;                     // sources per tile
constexpr int LOOP_BMAX = 64;                             // largest split
constexpr uint32_t LOOP_SPINS = 1u << 21;                 // barrier wait bound (~2 s)

// Barrier over the workgroups [f, f + W) of a cooperative launch: one
// arrival counter (bar[LOOP_FLAG * f], monotonic within a launch) and one
// generation word (bar[LOOP_FLAG * (f + 1)], its own 128-byte line).  Each
// workgroup releases its writes (agent-scope release fence) and adds 1 to the
// counter; the arrival that brings it to e W (epoch e, uint32 arithmetic,
// so it wraps consistently) acquires the others' writes and stores e into
// the generation word with release order; the others poll that word and
// acquire once it holds e or later.  One release and one acquire per
// workgroup and barrier: the fences (which write back / invalidate the
// XCD's L2) are what a barrier costs here, about 1.1 us at W = 16 and growing
// with W (measured: 3.3 us at W = 64, 11 us at 256, against 6.9 and 26 us
// for one flag per workgroup polled by every workgroup with two full fences
// each).  A wait longer than LOOP_SPINS polls sets ERR_LOOP and returns
// false (the workgroup then leaves the loop; the others follow at their next
// barrier), so no wave waits forever.  Epochs start at 1 in every launch;
// the host clears the words before it.
constexpr int LOOP_FLAG = 32;   // uint32 words per line
__device__ __forceinline__ bool group_sync(uint32_t *bar, uint32_t f, uint32_t W, uint32_t *err,
                                           uint32_t &epoch)
{
    if (W == 1) {
        __syncthreads();
        return true;
    }
    __shared__ int ok;
    const uint32_t e = ++epoch;
    __syncthreads();
    if (threadIdx.x == 0) {
        ok = 1;
        uint32_t *cnt = bar + LOOP_FLAG * f, *gen = bar + LOOP_FLAG * (f + 1);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t old = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        if (old == e * W - 1u) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(gen, e, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            uint32_t spins = 0;
            while ((int32_t)(__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) -
                             e) < 0) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > LOOP_SPINS) {
                    atomicOr(err, ERR_LOOP);
                    ok = 0;
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return ok != 0;
}

__device__ __forceinline__ bool grid_sync(uint32_t *bar, uint32_t nblk, uint32_t *err,
                                          uint32_t &epoch)
{
    return group_sync(bar, 0, nblk, err, epoch);
}

// minimum of t + dt over [b, e) (ordered bits) and how many reach it; the
// result is valid in thread 0
__device__ __forceinline__ void range_min_count(const double *t, const double *dt, int64_t b,
                                                int64_t e, uint64_t &v, int &cnt)
{
    __shared__ uint64_t rv[TPB / 64];
    __shared__ int rn[TPB / 64];
    v = ~0ull;
    cnt = 0;
    for (int64_t i = b + threadIdx.x; i < e; i += TPB)
        min_count(v, cnt, (uint64_t)__double_as_longlong(t[i] + dt[i]), 1);
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint64_t ov = __shfl_xor(v, m, 64);
        const int on = __shfl_xor(cnt, m, 64);
        min_count(v, cnt, ov, on);
    }
    if ((threadIdx.x & 63) == 0) {
        rv[threadIdx.x >> 6] = v;
        rn[threadIdx.x >> 6] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < TPB / 64; ++w)
            min_count(v, cnt, rv[w], rn[w]);
    __syncthreads();
}

// workgroup-wide minimum / sum, returned to every lane
__device__ __forceinline__ uint64_t block_min_u64(uint64_t v)
{
    __shared__ uint64_t r[TPB / 64];
    v = wave_min_u64(v);
    if ((threadIdx.x & 63) == 0)
        r[threadIdx.x >> 6] = v;
    __syncthreads();
    uint64_t m = r[0];
    for (int w = 1; w < TPB / 64; ++w)
        m = r[w] < m ? r[w] : m;
    __syncthreads();
    return m;
}

__device__ __forceinline__ int64_t block_sum_i64(int64_t v)
{
    __shared__ int64_t r[TPB / 64];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        v += __shfl_xor(v, m, 64);
    if ((threadIdx.x & 63) == 0)
        r[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t s = 0;
    for (int w = 0; w < TPB / 64; ++w)
        s += r[w];
    __syncthreads();
    return s;
}

template <int PREC>
__device__ __forceinline__ const typename Smem<PREC>::R &loop_records(const JRecMixed &jm,
                                                                      const JRecPair32 &jp,
                                                                      const JRecF64 &jd)
{
    if constexpr (std::is_same<typename Smem<PREC>::R, JRecMixed>::value)
        return jm;
    else if constexpr (std::is_same<typename Smem<PREC>::R, JRecPair32>::value)
        return jp;
    else
        return jd;
}

// A group's evaluation units (i-block u % n_ib against split u / n_ib).  A
// workgroup alone takes them in order (without a counter, workgroup r of W
// takes every W-th from r); in a group of several, each
// workgroup takes the next unit from the group's counter (*ctr, one atomic
// add per unit) until none is left, so that a workgroup slowed by its
// neighbours on the compute unit does not hold the others up.  The counter
// is never reset: each pass advances it by the units plus one failed take
// per workgroup, which every workgroup of the group adds to *base alike.
// Which workgroup evaluates a unit does not change its partial sums.
template <int PREC, bool EPS0, int LPI>
__device__ __forceinline__ void group_units(const typename Smem<PREC>::R &J, const ForceWork &w,
                                          double *part, int64_t n_act, double eps2, int64_t n_ib,
                                          int64_t B, int r, int W, uint32_t *ctr,
                                          uint32_t &base)
{
    const ForceOut none{};
    const int64_t units = n_ib * B;
    if (W == 1 || !ctr) {   // alone, or no counter: round-robin
        for (int64_t u = r; u < units; u += W)
            force_block<PREC, LPI, LOOP_NW, EPS0, false>(J, w, none, part, n_act, eps2, u % n_ib,
                                                          (int)(u / n_ib));
        return;
    }
    __shared__ uint32_t take;
    for (;;) {
        if (threadIdx.x == 0)
            take = atomicAdd(ctr, 1u) - base;
        __syncthreads();
        const int64_t u = take;
        __syncthreads();
        if (u >= units)
            break;
        force_block<PREC, LPI, LOOP_NW, EPS0, false>(J, w, none, part, n_act, eps2, u % n_ib,
                                                      (int)(u / n_ib));
    }
    base += (uint32_t)(units + W);
}

// res (mapped host memory): [0] block steps, [1] sum of N_act, [2] sum of
// N_act * n, [3] reason (LOOP_DONE, LOOP_BIG, LOOP_ERR), [4] N_act of the
// block it stopped at, then [7] = seq with system-scope release order.
template <int PREC, bool EPS0>
__global__ __launch_bounds__(TPB) void step_loop_kernel(
    State st, JRecMixed jm, JRecPair32 jp, JRecF64 jd, int prec, int64_t n, double eps2,
    double t_target,
    double eta, double dt_min, double dt_max, int64_t a_max, int32_t *act, double *part,
    int64_t *seg, const int64_t *off, uint64_t *wmin, int32_t *wcnt, uint32_t *bar,
    uint32_t *err, int64_t *hist, int64_t *res, int64_t seq)
{
    __shared__ double sum[9][RC_SLOTS];
    const auto &J = loop_records<PREC>(jm, jp, jd);
    const uint32_t G = gridDim.x;
    const int64_t P = (n + G - 1) / G;
    const int64_t r0 = (int64_t)blockIdx.x * P < n ? (int64_t)blockIdx.x * P : n;
    const int64_t r1 = r0 + P < n ? r0 + P : n;
    int64_t steps = 0, act_sum = 0, pairs = 0, stop_n = 0;
    int reason = 0;
    uint32_t epoch = 0;
    // unit counter (group_units): barrier line 2, or none for fewer than
    // three workgroups (only lines 0 and 1 are cleared then)
    uint32_t *uctr = G >= 3 ? bar + LOOP_FLAG * 2 : nullptr, ubase = 0;

    uint64_t v;
    int cnt;
    range_min_count(st.t, st.dt, r0, r1, v, cnt);
    if (threadIdx.x == 0) {
        wmin[blockIdx.x] = v;
        wcnt[blockIdx.x] = cnt;
    }
    for (;;) {
        if (!grid_sync(bar, G, err, epoch)) {
            reason = LOOP_ERR;
            break;
        }
        // (2) block time, N_act and this workgroup's offset, everywhere alike
        uint64_t tv = ~0ull;
        for (uint32_t w = threadIdx.x; w < G; w += TPB) {
            const uint64_t x = wmin[w];
            tv = x < tv ? x : tv;
        }
        const uint64_t T_bits = block_min_u64(tv);
        int64_t tot = 0, before = 0;
        for (uint32_t w = threadIdx.x; w < G; w += TPB)
            if (wmin[w] == T_bits) {
                tot += wcnt[w];
                before += w < blockIdx.x ? wcnt[w] : 0;
            }
        const int64_t n_act = block_sum_i64(tot);
        const int64_t first = block_sum_i64(before);
        const double T = __longlong_as_double((long long)T_bits);
        if (*(volatile uint32_t *)err != 0)
            reason = LOOP_ERR;
        else if (n_act == 0 || !(T <= t_target))
            reason = LOOP_DONE;
        else if (n_act > a_max)
            reason = LOOP_BIG;
        if (reason) {
            stop_n = n_act;
            break;
        }
        const int64_t mine = wmin[blockIdx.x] == T_bits ? (int64_t)wcnt[blockIdx.x] : 0;
        if (mine > 0)
            scatter_range(st.t, st.dt, T, r0, r1, first, act);
        pack_range(st, jm, jp, jd, prec, n, r0, r1, T);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            seg[0] = 0;
            seg[1] = n_act;
            int bb = 0;
            while ((int64_t(1) << (bb + 1)) <= n_act)
                ++bb;
            atomicAdd((unsigned long long *)&hist[bb], 1ull);
        }
        ++steps;
        act_sum += n_act;
        pairs += n_act * n;
        if (!grid_sync(bar, G, err, epoch)) {
            reason = LOOP_ERR;
            break;
        }
        // (3) evaluation units, shaped and taken as in the ensemble loop's
        // groups (the loop's workgroups are one group): 1, 8 or 32 lanes
        // per particle, then source splits for about four units per
        // workgroup, each workgroup taking the next unit from the counter in
        // the barrier line 2 (cleared with the others before the launch)
        const int64_t units = 4 * (int64_t)G;
        const int lpi = n_act >= (int64_t)TPB * G ? 1 : (n_act * 8 >= TPB ? 8 : 32);
        const int64_t ib = (int64_t)LOOP_NW * (64 / lpi);
        const int64_t n_ib = (n_act + ib - 1) / ib;
        int64_t B = 1;
        while (B * 2 <= LOOP_BMAX && B * n_ib < units && B * 2 * LOOP_NT <= n)
            B *= 2;
        ForceWork w{};
        w.idx = act;
        w.seg = seg;
        w.off = off;
        w.split = (int32_t)B;
        w.nc = 1;
        w.n_blocks = n_ib;
        if (lpi == 32)
            group_units<PREC, EPS0, 32>(J, w, part, n_act, eps2, n_ib, B, (int)blockIdx.x, (int)G,
                                        uctr, ubase);
        else if (lpi == 8)
            group_units<PREC, EPS0, 8>(J, w, part, n_act, eps2, n_ib, B, (int)blockIdx.x, (int)G,
                                       uctr, ubase);
        else
            group_units<PREC, EPS0, 1>(J, w, part, n_act, eps2, n_ib, B, (int)blockIdx.x, (int)G,
                                       uctr, ubase);
        if (!grid_sync(bar, G, err, epoch)) {
            reason = LOOP_ERR;
            break;
        }
        // (4) this range's active particles: split sums (fixed order) and
        // the corrector, RC_SLOTS particles per pass
        const int64_t bc = splits_used(n, B, LOOP_NT);
        const int q = threadIdx.x / RC_SLOTS, kl = threadIdx.x % RC_SLOTS;
        for (int64_t k0 = first; k0 < first + mine; k0 += RC_SLOTS) {
            const int64_t k = k0 + kl;
            const bool in = k < first + mine;
            const bool corr = threadIdx.x < RC_SLOTS && in;
            OldState o{};
            if (corr)
                o = load_old(st, n, act[k]);
            if (q < 9 && in)
                sum[q][kl] = sum_splits(part + (int64_t)q * n_act + k, 10 * n_act, bc);
            __syncthreads();
            if (corr) {
                const double a1[3] = {sum[0][kl], sum[1][kl], sum[2][kl]};
                const double j1[3] = {sum[3][kl], sum[4][kl], sum[5][kl]};
                const double s1[3] = {sum[6][kl], sum[7][kl], sum[8][kl]};
                correct_loaded(st, n, act[k], o, a1, j1, s1, t_target, eta, dt_min, dt_max,
                               err);
            }
            __syncthreads();
        }
        // (1) of the next step, over the range this workgroup just updated
        range_min_count(st.t, st.dt, r0, r1, v, cnt);
        if (threadIdx.x == 0) {
            wmin[blockIdx.x] = v;
            wcnt[blockIdx.x] = cnt;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        res[0] = steps;
        res[1] = act_sum;
        res[2] = pairs;
        res[3] = reason;
        res[4] = stop_n;
        __hip_atomic_store(&res[7], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// --------------------------------------------------- ensemble block steps
// Independent clusters advanced to t_target in one persistent launch: the
// workgroups form groups (EnsPlan: group g holds the W_g consecutive
// workgroups from first[g] and integrates the clusters cl[cl_off[g] ..
// cl_off[g+1]) one after another).  For each cluster the group runs the
// block steps of step_loop_kernel restricted to the cluster's particles,
// with its barriers restricted to the group (a group of one workgroup needs
// only workgroup barriers), its active list at act[o0 ..) and its split
// partials in the group's own part region [part_off[g], + part_cap[g])
// slots.  Clusters never interact, so no barrier spans the chip.  The
// evaluation shape follows N_act and the group size (1, 8 or 32 lanes per
// particle, then source splits, for about four units per workgroup of a
// group).  Per-workgroup minima and counts are kept in two
// banks by cluster parity: a workgroup that has finished a cluster may start
// the next while a slower one still reads the last decision's values.
// res (device): [0] sum of N_act, [1] sum of N_act * N_c, [2] largest number
// of block steps of a cluster (the number of batched block steps of the
// host-sized path)
template <int PREC, bool EPS0>
__global__ __launch_bounds__(TPB, 4) void ensemble_loop_kernel(
    State st, JRecMixed jm, JRecPair32 jp, JRecF64 jd, int prec, int64_t n, double eps2,
    double t_target, double eta, double dt_min, double dt_max, int32_t *act, double *part,
    const int64_t *off, EnsPlan plan, uint64_t *wmin, int32_t *wcnt, uint32_t *bar,
    uint32_t *err, int64_t *hist, unsigned long long *res)
{
    __shared__ double sum[9][RC_SLOTS];
    const auto &J = loop_records<PREC>(jm, jp, jd);
    const int g = plan.grp_of[blockIdx.x];
    const uint32_t f = (uint32_t)plan.first[g], W = (uint32_t)plan.size[g];
    const int r = (int)(blockIdx.x - f);
    int64_t *seg = plan.seg + 2 * g;
    double *gpart = part + plan.part_off[g] * 10;
    const int64_t cap = plan.part_cap[g];
    uint32_t epoch = 0;
    // the group's unit counter: its own 128-byte line after the barrier lines
    uint32_t *uctr = bar + LOOP_BAR_WORDS + LOOP_FLAG * g, ubase = 0;
    int64_t act_sum = 0, pairs = 0, steps_max = 0;
    bool failed = false;
    for (int q = plan.cl_off[g]; q < plan.cl_off[g + 1] && !failed; ++q) {
        const int c = plan.cl[q];
        const int64_t o0 = off[c], o1 = off[c + 1], nc_ = o1 - o0;
        const int64_t P = (nc_ + W - 1) / W;
        const int64_t r0 = o0 + ((int64_t)r * P < nc_ ? (int64_t)r * P : nc_);
        const int64_t r1 = r0 + P < o1 ? r0 + P : o1;
        int32_t *act_c = act + o0;
        uint64_t *wm = wmin + (q & 1) * LOOP_GMAX;
        int32_t *wc = wcnt + (q & 1) * LOOP_GMAX;
        int64_t steps = 0;
        uint64_t v;
        int cnt;
        range_min_count(st.t, st.dt, r0, r1, v, cnt);
        if (threadIdx.x == 0) {
            wm[blockIdx.x] = v;
            wc[blockIdx.x] = cnt;
        }
        for (;;) {
            if (!group_sync(bar, f, W, err, epoch)) {
                failed = true;
                break;
            }
            // (2) block time, N_act and this workgroup's offset, alike in the group
            uint64_t tv = ~0ull;
            for (uint32_t k = threadIdx.x; k < W; k += TPB) {
                const uint64_t x = wm[f + k];
                tv = x < tv ? x : tv;
            }
            const uint64_t T_bits = block_min_u64(tv);
            int64_t tot = 0, before = 0;
            for (uint32_t k = threadIdx.x; k < W; k += TPB)
                if (wm[f + k] == T_bits) {
                    tot += wc[f + k];
                    before += (int)k < r ? wc[f + k] : 0;
                }
            const int64_t n_act = block_sum_i64(tot);
            const int64_t first = block_sum_i64(before);
            const double T = __longlong_as_double((long long)T_bits);
            if (*(volatile uint32_t *)err != 0) {
                failed = true;
                break;
            }
            if (n_act == 0 || !(T <= t_target))
                break;
            const int64_t mine = wm[blockIdx.x] == T_bits ? (int64_t)wc[blockIdx.x] : 0;
            if (mine > 0)
                scatter_range(st.t, st.dt, T, r0, r1, first, act_c);
            // one particle per lane and pass: the kernel is held to 128
            // registers, and two in flight would spill
            for (int64_t i = r0 + threadIdx.x; i < r1; i += TPB)
                pack_h(st, jm, jp, jd, prec, n, i, T - st.t[i]);
            if (r == 0 && threadIdx.x == 0) {
                seg[0] = 0;
                seg[1] = n_act;
                int bb = 0;
                while ((int64_t(1) << (bb + 1)) <= n_act)
                    ++bb;
                atomicAdd((unsigned long long *)&hist[bb], 1ull);
            }
            ++steps;
            act_sum += n_act;
            pairs += n_act * nc_;
            if (!group_sync(bar, f, W, err, epoch)) {
                failed = true;
                break;
            }
            // (3) evaluation units of the group: i-blocks against source
            // splits.  Lanes per particle: 1 when the active particles give
            // every lane of the group one, else 8 when they fill one
            // workgroup's lanes, else 32 (fewer lanes per particle mean
            // more pairs per lane and LDS tile, so the tile loads and lane
            // reductions cost less per pair).  Then source splits until a
            // group of several has about four units per workgroup (a
            // workgroup alone takes the block in as few units as possible).
            const int64_t units = W == 1 ? 1 : 4 * (int64_t)W;
            const int lpi = n_act >= (int64_t)TPB * W ? 1 : (n_act * 8 >= TPB ? 8 : 32);
            const int64_t ib = (int64_t)LOOP_NW * (64 / lpi);
            const int64_t n_ib = (n_act + ib - 1) / ib;
            int64_t B = 1;
            while (B * 2 <= LOOP_BMAX && B * n_ib < units && B * 2 * LOOP_NT <= nc_ &&
                   B * 2 * n_act <= cap)
                B *= 2;
            ForceWork w{};
            w.idx = act_c;
            w.seg = seg;
            w.off = off + c;
            w.split = (int32_t)B;
            w.nc = 1;
            w.n_blocks = n_ib;
            if (lpi == 32)
                group_units<PREC, EPS0, 32>(J, w, gpart, n_act, eps2, n_ib, B, r, (int)W, uctr,
                                          ubase);
            else if (lpi == 8)
                group_units<PREC, EPS0, 8>(J, w, gpart, n_act, eps2, n_ib, B, r, (int)W, uctr,
                                         ubase);
            else
                group_units<PREC, EPS0, 1>(J, w, gpart, n_act, eps2, n_ib, B, r, (int)W, uctr,
                                         ubase);
            if (!group_sync(bar, f, W, err, epoch)) {
                failed = true;
                break;
            }
            // (4) this workgroup's active particles: split sums (fixed order)
            // and the corrector, RC_SLOTS particles per pass
            const int64_t bc = splits_used(nc_, B, LOOP_NT);
            const int qq = threadIdx.x / RC_SLOTS, kl = threadIdx.x % RC_SLOTS;
            for (int64_t k0 = first; k0 < first + mine; k0 += RC_SLOTS) {
                const int64_t k = k0 + kl;
                const bool in = k < first + mine;
                const bool corr = threadIdx.x < RC_SLOTS && in;
                OldState o{};
                if (corr)
                    o = load_old(st, n, act_c[k]);
                if (qq < 9 && in)
                    sum[qq][kl] = sum_splits(gpart + (int64_t)qq * n_act + k, 10 * n_act, bc);
                __syncthreads();
                if (corr) {
                    const double a1[3] = {sum[0][kl], sum[1][kl], sum[2][kl]};
                    const double j1[3] = {sum[3][kl], sum[4][kl], sum[5][kl]};
                    const double s1[3] = {sum[6][kl], sum[7][kl], sum[8][kl]};
                    correct_loaded(st, n, act_c[k], o, a1, j1, s1, t_target, eta, dt_min,
                                   dt_max, err);
                }
                __syncthreads();
            }
            // (1) of the next step, over the range this workgroup just updated
            range_min_count(st.t, st.dt, r0, r1, v, cnt);
            if (threadIdx.x == 0) {
                wm[blockIdx.x] = v;
                wc[blockIdx.x] = cnt;
            }
        }
        steps_max = steps > steps_max ? steps : steps_max;
    }
    if (r == 0 && threadIdx.x == 0) {
        atomicAdd(&res[0], (unsigned long long)act_sum);
        atomicAdd(&res[1], (unsigned long long)pairs);
        atomicMax(&res[2], (unsigned long long)steps_max);
    }
}

// first step after the start-up evaluation: the generalized criterion at
// the order the known derivatives allow (p = 4), eta_init A(1) / A(2)
__global__ __launch_bounds__(TPB) void init_dt_kernel(State st, int64_t n, double eta_init,
                                                      double dt_min, double dt_max,
                                                      uint32_t *err)
{
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n)
        return;
    const double na = norm3(st.acc[i], st.acc[n + i], st.acc[2 * n + i]);
    const double nj = norm3(st.jrk[i], st.jrk[n + i], st.jrk[2 * n + i]);
    const double ns = norm3(st.snp[i], st.snp[n + i], st.snp[2 * n + i]);
    const double nc = norm3(st.crk[i], st.crk[n + i], st.crk[2 * n + i]);
    const double A1 = sqrt(na * ns + nj * nj);
    const double A2 = sqrt(nj * nc + ns * ns);
    const double crit = A2 > 0.0 ? eta_init * A1 / A2 : INFINITY;
    double dt = dt_max;
    const uint32_t bad = block_dt(crit, 0.0, 0.0, INFINITY, dt_min, dt_max, &dt);
    st.dt[i] = dt;
    st.t[i] = 0.0;
    if (bad)
        atomicOr(err, bad);
}

// start of a run: a particle short of t_target whose step passes it halves
// the step until it does not; a particle past t_target is an error
__global__ __launch_bounds__(TPB) void recap_kernel(State st, int64_t n, double t_target,
                                                    uint32_t *err)
{
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n)
        return;
    const double t = st.t[i];
    double dt = st.dt[i];
    if (t > t_target) {
        atomicOr(err, ERR_BADIDX);
        return;
    }
    if (t < t_target) {
        for (int it = 0; it < 80 && t + dt > t_target; ++it)
            dt *= 0.5;
        st.dt[i] = dt;
    }
}

// ------------------------------------------------------------- energy
// per-workgroup partial sums of E_kin, sum_i m_i phi_i (phi_i over j > i,
// so each pair once), L; then one workgroup adds the partials in order
__device__ __forceinline__ double block_sum(double v, double *sh)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        v += __shfl_xor(v, m, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
        s += sh[w];
    return s;
}

__global__ __launch_bounds__(TPB) void energy_partial(State st, int64_t n, const double *phi,
                                                      double *red)
{
    __shared__ double sh[TPB / 64];
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    double q[5] = {0, 0, 0, 0, 0};
    if (i < n) {
        const double m = st.mass[i];
        const double x = st.pos[i], y = st.pos[n + i], z = st.pos[2 * n + i];
        const double vx = st.vel[i], vy = st.vel[n + i], vz = st.vel[2 * n + i];
        q[0] = 0.5 * m * (vx * vx + vy * vy + vz * vz);
        q[1] = m * phi[i];   // phi[i] = -sum of m_j / r_ij over the half-window of i
        q[2] = m * (y * vz - z * vy);
        q[3] = m * (z * vx - x * vz);
        q[4] = m * (x * vy - y * vx);
    }
    for (int r = 0; r < 5; ++r) {
        const double s = block_sum(q[r], sh);
        if (threadIdx.x == 0)
            red[(int64_t)blockIdx.x * 5 + r] = s;
    }
}

__global__ __launch_bounds__(1024) void energy_final(const double *red, int64_t nblk,
                                                     double *out)
{
    __shared__ double sh[1024 / 64];
    for (int r = 0; r < 5; ++r) {
        double v = 0.0;
        for (int64_t b = threadIdx.x; b < nblk; b += 1024)
            v += red[b * 5 + r];
        const double s = block_sum(v, sh);
        if (threadIdx.x == 0)
            out[r] = s;
    }
}

// ------------------------------------------------------------ utilities
__global__ void validate_idx_kernel(const int32_t *idx, int64_t n_act, int64_t n, uint32_t *err)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_act)
        return;
    const int32_t i = idx[k];
    if (i < 0 || i >= n || (k > 0 && idx[k - 1] >= i))
        atomicOr(err, ERR_BADIDX);
}

// Energy precondition: every particle of a cluster at the cluster's first
// particle's time (the sums of paper Sect. 5.1 are taken at a common time).
__global__ void sync_check_kernel(const double *t, int64_t n, const int32_t *cluster_of,
                                  const int64_t *off, uint32_t *err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int c = cluster_of ? cluster_of[i] : 0;
    if (t[i] != t[off[c]])
        atomicOr(err, ERR_STATE);
}

__global__ void aos_to_soa_kernel(const double *src, double *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    dst[i] = src[3 * i];
    dst[n + i] = src[3 * i + 1];
    dst[2 * n + i] = src[3 * i + 2];
}

__global__ void soa_to_aos_kernel(const double *src, double *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    dst[3 * i] = src[i];
    dst[3 * i + 1] = src[n + i];
    dst[3 * i + 2] = src[2 * n + i];
}

__global__ void check_finite_kernel(State st, int64_t n, uint32_t *err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    bool ok = isfinite(st.mass[i]);
    for (int d = 0; d < 3; ++d)
        ok = ok && isfinite(st.pos[(int64_t)d * n + i]) && isfinite(st.vel[(int64_t)d * n + i]);
    if (!ok)
        atomicOr(err, ERR_NONFINITE);
}

unsigned nblk(int64_t n, int t = TPB) { return (unsigned)((n + t - 1) / t); }

// Source records straight from caller arrays (mass[n], pos/vel/acc [n][3]
// row-major), at their own time: the records nbody_force builds from a
// context's stored state, for the evaluation that keeps no context.  Also
// writes the one-cluster work tables seg = {0, n_act}, off = {0, n}.
__global__ __launch_bounds__(TPB) void pack_arrays_kernel(const double *mass, const double *pos,
                                                          const double *vel, const double *acc,
                                                          JRecMixed jm, JRecPair32 jp, JRecF64 jd,
                                                          int prec, int64_t n, int64_t n_act,
                                                          int64_t *seg, int64_t *off)
{
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i == 0) {
        seg[0] = 0;
        seg[1] = n_act;
        off[0] = 0;
        off[1] = n;
    }
    if (i >= n)
        return;
    const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    const double vx = vel[3 * i], vy = vel[3 * i + 1], vz = vel[3 * i + 2];
    const double ax = acc[3 * i], ay = acc[3 * i + 1], az = acc[3 * i + 2];
    if (prec == NBODY_PREC_MIXED) {
        jm.x[i] = x; jm.y[i] = y; jm.z[i] = z; jm.m[i] = mass[i];
        jm.vx[i] = vx; jm.vy[i] = vy; jm.vz[i] = vz;
        jm.ax[i] = (float)ax; jm.ay[i] = (float)ay; jm.az[i] = (float)az;
    } else if (prec == NBODY_PREC_FP32PAIR) {
        jp.x[i] = x; jp.y[i] = y; jp.z[i] = z; jp.m[i] = mass[i];
        jp.vx[i] = (float)vx; jp.vy[i] = (float)vy; jp.vz[i] = (float)vz;
        jp.ax[i] = (float)ax; jp.ay[i] = (float)ay; jp.az[i] = (float)az;
    } else {
        jd.x[i] = x; jd.y[i] = y; jd.z[i] = z; jd.m[i] = mass[i];
        jd.vx[i] = vx; jd.vy[i] = vy; jd.vz[i] = vz;
        jd.ax[i] = ax; jd.ay[i] = ay; jd.az[i] = az;
    }
}

}  // namespace

hipError_t launch_pack_arrays(const Ctx &c, const double *mass, const double *pos,
                              const double *vel, const double *acc, int64_t n_act,
                              int64_t *seg, int64_t *off, hipStream_t s)
{
    hipLaunchKernelGGL(pack_arrays_kernel, dim3(nblk(c.n)), dim3(TPB), 0, s, mass, pos, vel, acc,
                       c.jm, c.jp, c.jd, (int)c.cfg.precision, c.n, n_act, seg, off);
    return hipGetLastError();
}

hipError_t launch_pack(const Ctx &c, const double *T_cluster, int own_time,
                       const int32_t *cluster_of, hipStream_t s)
{
    hipLaunchKernelGGL(pack_kernel, dim3(nblk(c.n)), dim3(TPB), 0, s, c.st, c.jm, c.jp, c.jd,
                       (int)c.cfg.precision, c.n, T_cluster, cluster_of, own_time);
    return hipGetLastError();
}

hipError_t launch_predict_out(const Ctx &c, double t, double *pos, double *vel, double *acc,
                              hipStream_t s)
{
    hipLaunchKernelGGL(predict_out_kernel, dim3(nblk(c.n)), dim3(TPB), 0, s, c.st, c.n, t,
                       pos, vel, acc);
    return hipGetLastError();
}

hipError_t launch_sched_reset(const Ctx &c, hipStream_t s)
{
    hipLaunchKernelGGL(sched_reset, dim3(nblk(c.nc)), dim3(TPB), 0, s, c.d_tmin, c.nc);
    return hipGetLastError();
}

// minima, counts and scan: block times, segments, N_act (info) -- the
// per-cluster minima must be reset (at init, and by every scan after use)
hipError_t launch_sched_head(const Ctx &c, double t_target, int64_t seq, hipStream_t s)
{
    hipLaunchKernelGGL(sched_min, dim3((unsigned)c.n_chunks), dim3(TPB), 0, s,
                       (const double *)c.st.t, (const double *)c.st.dt,
                       (const int64_t *)c.d_chunk_begin, (const int32_t *)c.d_chunk_cluster,
                       c.d_tmin, c.d_chunk_min, c.d_chunk_cnt);
    hipLaunchKernelGGL(sched_scan, dim3(1), dim3(1024), 0, s, (const uint64_t *)c.d_chunk_min,
                       (const int32_t *)c.d_chunk_cnt, c.n_chunks,
                       (const int32_t *)c.d_chunk_cluster, c.d_tmin, (const int64_t *)c.d_off,
                       c.nc, t_target, c.d_chunk_pos, c.d_seg, c.d_tblock, c.d_info,
                       c.d_info + 8, (const uint32_t *)c.d_err, c.d_tot, seq);
    return hipGetLastError();
}

// compaction of the active list and predictor of a block step, one launch
hipError_t launch_scatter_pack(const Ctx &c, hipStream_t s, bool levels)
{
    const unsigned nb = (unsigned)c.n_chunks + nblk(c.n);
    hipLaunchKernelGGL(scatter_pack_kernel, dim3(nb), dim3(TPB), 0, s, c.st, c.jm, c.jp, c.jd,
                       (int)c.cfg.precision, c.n, (const int32_t *)c.d_cluster_of,
                       (const int64_t *)c.d_chunk_begin, (const int32_t *)c.d_chunk_cluster,
                       (const double *)c.d_tblock, (const int64_t *)c.d_chunk_pos, c.act,
                       c.n_chunks, levels ? c.d_lvl + LVL_POS : (int64_t *)nullptr);
    return hipGetLastError();
}

// per-level counts of the stored state (see levels_build_kernel)
hipError_t launch_levels_build(const Ctx &c, hipStream_t s)
{
    hipError_t e = hipMemsetAsync(c.d_lvl, 0, LVL_WORDS * sizeof(int64_t), s);
    if (e != hipSuccess)
        return e;
    const int e0 = std::ilogb(c.cfg.dt_max), e1 = std::ilogb(c.cfg.dt_min);
    hipLaunchKernelGGL(levels_build_kernel, dim3(nblk(c.n)), dim3(TPB), 0, s,
                       (const double *)c.st.t, (const double *)c.st.dt, c.n, e0, e0 - e1,
                       c.d_lvl);
    hipLaunchKernelGGL(levels_check_kernel, dim3(nblk(c.n)), dim3(TPB), 0, s,
                       (const double *)c.st.t, (const double *)c.st.dt, c.n, c.d_lvl);
    return hipGetLastError();
}

hipError_t launch_levels_sched(const Ctx &c, double t_target, int64_t seq, hipStream_t s)
{
    hipLaunchKernelGGL(levels_sched_kernel, dim3(1), dim3(64), 0, s, c.d_lvl, c.n,
                       std::ilogb(c.cfg.dt_max), t_target, c.d_seg, c.d_tblock, c.d_info,
                       c.d_info + 8, c.d_err, c.d_tot, seq);
    return hipGetLastError();
}

// ordered list of the due particles
hipError_t launch_sched_scatter(const Ctx &c, hipStream_t s)
{
    hipLaunchKernelGGL(sched_scatter, dim3((unsigned)c.n_chunks), dim3(TPB), 0, s,
                       (const double *)c.st.t, (const double *)c.st.dt,
                       (const int64_t *)c.d_chunk_begin, (const int32_t *)c.d_chunk_cluster,
                       (const double *)c.d_tblock, (const int64_t *)c.d_chunk_pos, c.act);
    return hipGetLastError();
}

hipError_t launch_schedule(const Ctx &c, double t_target, int64_t seq, hipStream_t s)
{
    hipError_t e = launch_sched_head(c, t_target, seq, s);
    return e != hipSuccess ? e : launch_sched_scatter(c, s);
}

namespace {

// the loop kernel for a context's precision and softening
const void *step_loop_fn(const Ctx &c)
{
    const bool e0 = c.eps == 0.0;
    switch (c.cfg.precision) {
    case NBODY_PREC_FP64:
        return e0 ? (const void *)step_loop_kernel<PREC_F64, true>
                  : (const void *)step_loop_kernel<PREC_F64, false>;
    case NBODY_PREC_FP32PAIR:
        return e0 ? (const void *)step_loop_kernel<PREC_PAIR32, true>
                  : (const void *)step_loop_kernel<PREC_PAIR32, false>;
    default:
        return e0 ? (const void *)step_loop_kernel<PREC_MIXED, true>
                  : (const void *)step_loop_kernel<PREC_MIXED, false>;
    }
}

// the ensemble loop kernel for a context's precision and softening
const void *ensemble_loop_fn(const Ctx &c)
{
    const bool e0 = c.eps == 0.0;
    switch (c.cfg.precision) {
    case NBODY_PREC_FP64:
        return e0 ? (const void *)ensemble_loop_kernel<PREC_F64, true>
                  : (const void *)ensemble_loop_kernel<PREC_F64, false>;
    case NBODY_PREC_FP32PAIR:
        return e0 ? (const void *)ensemble_loop_kernel<PREC_PAIR32, true>
                  : (const void *)ensemble_loop_kernel<PREC_PAIR32, false>;
    default:
        return e0 ? (const void *)ensemble_loop_kernel<PREC_MIXED, true>
                  : (const void *)ensemble_loop_kernel<PREC_MIXED, false>;
    }
}

}  // namespace

int ensemble_max_grid(const Ctx &c)
{
    int dev = 0, coop = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ensemble_loop_fn(c), TPB, 0) !=
            hipSuccess)
        return 0;
    if (!coop || per_cu < 1 || cus < 1)
        return 0;
    const int64_t g = (int64_t)per_cu * cus;
    return g < LOOP_GMAX ? (int)g : LOOP_GMAX;
}

// The ensemble's block steps to t_target in one launch (see
// ensemble_loop_kernel).  The caller has reset the barrier words and res,
// and filled the plan's tables; grid <= ensemble_max_grid(c).
hipError_t launch_ensemble_loop(const Ctx &c, double t_target, int grid, const EnsPlan &plan,
                                unsigned long long *res, hipStream_t s)
{
    State st = c.st;
    JRecMixed jm = c.jm;
    JRecPair32 jp = c.jp;
    JRecF64 jd = c.jd;
    int prec = c.cfg.precision;
    int64_t n = c.n;
    double eps2 = c.eps * c.eps, tt = t_target, eta = c.cfg.eta, dmin = c.cfg.dt_min,
           dmax = c.cfg.dt_max;
    int32_t *act = c.act;
    double *part = c.part;
    const int64_t *off = c.d_off;
    EnsPlan pl = plan;
    uint64_t *wmin = c.d_loop_min;
    int32_t *wcnt = c.d_loop_cnt;
    uint32_t *bar = c.d_loop_bar;
    uint32_t *err = c.d_err;
    int64_t *hist = c.d_info + 8;
    unsigned long long *r = res;
    void *args[] = {&st,  &jm,   &jp,  &jd,  &prec, &n,    &eps2, &tt,  &eta, &dmin,
                    &dmax, &act, &part, &off, &pl,   &wmin, &wcnt, &bar, &err, &hist, &r};
    return hipLaunchCooperativeKernel(ensemble_loop_fn(c), dim3((unsigned)grid), dim3(TPB), args,
                                      0, s);
}

int step_loop_max_grid(const Ctx &c)
{
    int dev = 0, coop = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, step_loop_fn(c), TPB, 0) !=
            hipSuccess)
        return 0;
    if (!coop || per_cu < 1 || cus < 1)
        return 0;
    // one workgroup per compute unit: more would only lengthen the barriers
    return cus < LOOP_GMAX ? cus : LOOP_GMAX;
}

// Device-resident block steps (see step_loop_kernel).  The caller has reset
// the barrier words; grid <= step_loop_max_grid(c).
hipError_t launch_step_loop(const Ctx &c, double t_target, int64_t a_max, int grid, int64_t seq,
                            hipStream_t s)
{
    State st = c.st;
    JRecMixed jm = c.jm;
    JRecPair32 jp = c.jp;
    JRecF64 jd = c.jd;
    int prec = c.cfg.precision;
    int64_t n = c.n;
    double eps2 = c.eps * c.eps, tt = t_target, eta = c.cfg.eta, dmin = c.cfg.dt_min,
           dmax = c.cfg.dt_max;
    int64_t am = a_max, sq = seq;
    int32_t *act = c.act;
    double *part = c.part;
    int64_t *seg = c.d_seg;
    const int64_t *off = c.d_off;
    uint64_t *wmin = c.d_loop_min;
    int32_t *wcnt = c.d_loop_cnt;
    uint32_t *bar = c.d_loop_bar;
    uint32_t *err = c.d_err;
    int64_t *hist = c.d_info + 8;
    int64_t *res = c.d_tot + 8;
    void *args[] = {&st,   &jm,  &jp,  &jd,   &prec, &n,    &eps2, &tt,  &eta,  &dmin, &dmax, &am,
                    &act,  &part, &seg, &off,  &wmin, &wcnt, &bar, &err,  &hist, &res,  &sq};
    return hipLaunchCooperativeKernel(step_loop_fn(c), dim3((unsigned)grid), dim3(TPB), args, 0,
                                      s);
}

hipError_t launch_blocks(const Ctx &c, int64_t ib, int64_t cap, hipStream_t s)
{
    hipLaunchKernelGGL(blocks_kernel, dim3(1), dim3(1024), 0, s, (const int64_t *)c.d_seg,
                       c.nc, ib, cap, c.d_blk_first, c.d_blk_cluster);
    return hipGetLastError();
}

hipError_t launch_segments(const Ctx &c, const int32_t *idx, int64_t n_act, hipStream_t s)
{
    if (c.nc == 1 && idx) {
        hipLaunchKernelGGL(set_seg_kernel, dim3(1), dim3(1), 0, s, c.d_seg, (int64_t)0, n_act);
    } else {
        hipLaunchKernelGGL(segments_kernel, dim3(nblk(c.nc + 1)), dim3(TPB), 0, s, idx, n_act,
                           (const int64_t *)c.d_off, c.nc, c.d_seg);
    }
    return hipGetLastError();
}

hipError_t launch_correct(const Ctx &c, int64_t n_act, const int32_t *idx, double t_target,
                          const double *fa, const double *fj, const double *fs, int64_t sk,
                          int64_t sd, hipStream_t s, bool levels)
{
    if (n_act <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(correct_kernel, dim3(nblk(n_act)), dim3(TPB), 0, s, c.st, c.n, n_act,
                       idx, t_target, fa, fj, fs, sk, sd, c.cfg.eta, c.cfg.dt_min,
                       c.cfg.dt_max, c.d_err, levels ? c.d_lvl : nullptr,
                       std::ilogb(c.cfg.dt_max));
    return hipGetLastError();
}

hipError_t launch_reduce_correct(const Ctx &c, const ForceWork &w, int split, int nt,
                                 int64_t n_act, double t_target, hipStream_t s, bool levels)
{
    if (n_act <= 0)
        return hipSuccess;
    // lanes per sum by the number of splits (chains of at most ~32 loads)
    const int R = split <= 32 ? 1 : (split <= 128 ? 4 : 8);
    const int S = TPB / (9 * R);
    const unsigned nb = (unsigned)((n_act + S - 1) / S);
    auto k = R == 1 ? reduce_correct_kernel<1> : (R == 4 ? reduce_correct_kernel<4>
                                                           : reduce_correct_kernel<8>);
    hipLaunchKernelGGL(k, dim3(nb), dim3(TPB), 0, s, c.st, c.n, n_act,
                       (const double *)c.part, (int32_t)split, nt, w,
                       (const int32_t *)c.d_cluster_of, t_target, c.cfg.eta, c.cfg.dt_min,
                       c.cfg.dt_max, c.d_err, levels ? c.d_lvl : nullptr,
                       std::ilogb(c.cfg.dt_max));
    return hipGetLastError();
}

hipError_t launch_recap(const Ctx &c, double t_target, hipStream_t s)
{
    hipLaunchKernelGGL(recap_kernel, dim3(nblk(c.n)), dim3(TPB), 0, s, c.st, c.n, t_target,
                       c.d_err);
    return hipGetLastError();
}

hipError_t launch_init_dt(const Ctx &c, hipStream_t s)
{
    hipLaunchKernelGGL(init_dt_kernel, dim3(nblk(c.n)), dim3(TPB), 0, s, c.st, c.n,
                       c.cfg.eta_init, c.cfg.dt_min, c.cfg.dt_max, c.d_err);
    return hipGetLastError();
}

hipError_t launch_energy_sums(const Ctx &c, const double *phi, double *out5, hipStream_t s)
{
    const unsigned nb = nblk(c.n);
    hipLaunchKernelGGL(energy_partial, dim3(nb), dim3(TPB), 0, s, c.st, c.n, phi, c.d_red);
    hipLaunchKernelGGL(energy_final, dim3(1), dim3(1024), 0, s, (const double *)c.d_red,
                       (int64_t)nb, out5);
    return hipGetLastError();
}

hipError_t launch_validate_idx(const Ctx &c, int64_t n_act, const int32_t *idx, hipStream_t s)
{
    if (n_act <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(validate_idx_kernel, dim3(nblk(n_act)), dim3(TPB), 0, s, idx, n_act,
                       c.n, c.d_err);
    return hipGetLastError();
}

hipError_t launch_sync_check(const Ctx &c, hipStream_t s)
{
    hipLaunchKernelGGL(sync_check_kernel, dim3(nblk(c.n)), dim3(TPB), 0, s,
                       (const double *)c.st.t, c.n, (const int32_t *)c.d_cluster_of,
                       (const int64_t *)c.d_off, c.d_err);
    return hipGetLastError();
}

hipError_t launch_aos_to_soa(const double *src, double *dst, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(aos_to_soa_kernel, dim3(nblk(n)), dim3(TPB), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_soa_to_aos(const double *src, double *dst, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(soa_to_aos_kernel, dim3(nblk(n)), dim3(TPB), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_check_finite(const Ctx &c, hipStream_t s)
{
    hipLaunchKernelGGL(check_finite_kernel, dim3(nblk(c.n)), dim3(TPB), 0, s, c.st, c.n,
                       c.d_err);
    return hipGetLastError();
}

}  // namespace nb
