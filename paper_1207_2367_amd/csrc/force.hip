// Evaluation step of the Hermite scheme on gfx950: acceleration, jerk, snap
// and potential of the active particles against all sources of their
// cluster (paper Sect. 3, item 2, with the softened potential of Sect. 2),
// plus the split-source reduction (the paper's "Bfactor", Sect. 3).
//
// Design (CDNA4, wave64):
//   - one workgroup = NW waves; each wave holds GI = 64 / LPI active
//     particles, LPI lanes per particle; the i-particle lives in registers;
//   - sources are staged through LDS in tiles of NT = 64 NW records (one
//     16-byte aligned record per source), loaded coalesced from the
//     structure-of-arrays source arrays by the whole workgroup; lane slot js
//     of an i-particle takes tile entries js, js + LPI, ...; with LPI = 1
//     every LDS read is a broadcast;
//   - the pair loop is pure vector ALU: no matrix cores, the work is not a
//     dense contraction (every pair needs a reciprocal square root and
//     nonlinear terms);
//   - mixed precision: r_j - r_i, r^2 and 1/r (v_rsq_f32 seed + one FP64
//     Newton step) in FP64, and with them the acceleration, jerk (from FP64
//     velocity differences) and potential terms, summed in FP64; the snap
//     term in FP32 from the rounded r_j - r_i, jerk vector and coefficients
//     and the FP32 acceleration differences, summed over at most 64 pairs
//     per lane in FP32 and folded into double-single (hi, lo) accumulators
//     by an error-free two-sum.  Per-term FP32 rounding in a sum with
//     cancellation grows with the sum's condition number, so the quantities
//     held to 1e-6 per particle (acceleration, jerk, potential) stay FP64;
//     the snap is the least amplified: the fifth-derivative estimate of the
//     step criterion multiplies the acceleration's absolute error by
//     ~720/h^5 but the snap's by at most ~1/h^3;
//   - the LPI lanes of a particle are combined by a xor butterfly of wave
//     shuffles (bitwise identical on every lane, fixed order);
//   - the FP64 passes take 1/r from the same FP32 seed, refined to FP64
//     accuracy by one third-order step;
//   - the potential energy (energy_kernel) takes every pair once, with a
//     cyclic half-window per particle that gives every workgroup equal work;
//   - grid.y = B splits the sources (chunks of whole tiles; a cluster with
//     fewer tiles uses fewer splits, the rest exit at once); partial results
//     go to a [B][10][n_act] buffer that a second kernel sums in fixed order
//     b = 0 .. B_c-1 (reduce_split here, the corrector's kernel in a block
//     step, or the correction phase of the device-resident loop), so the
//     result does not depend on scheduling (no float atomics anywhere);
//   - the per-workgroup body (force_block) lives in force_body.h, shared by
//     the launch kernel here and the device-resident block-step loop;
//   - a block step's evaluation skips the potential (template flag PHI).
#include "force_body.h"

namespace nb {

namespace {

// Potential terms of one LDS tile of NT sources for one lane: phi -= m_j /
// r_ij, FP64.  MASK keeps only the tile slots lo <= t <= hi.
template <int NT, bool MASK, bool EPS0>
__device__ __forceinline__ double pot_tile(const double *sx, const double *sy,
                                           const double *sz, const double *sm,
                                           double xi, double yi, double zi, double eps2,
                                           int lo, int hi, double phi)
{
#pragma unroll 8
    for (int t = 0; t < NT; ++t) {
        const double dx = sx[t] - xi, dy = sy[t] - yi, dz = sz[t] - zi;
        const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
        double rinv = rinv_f64(r2);
        if constexpr (EPS0)
            rinv = r2 > 0.0 ? rinv : 0.0;
        if constexpr (MASK)
            rinv = (t >= lo && t <= hi) ? rinv : 0.0;
        phi = fma(-sm[t], rinv, phi);
    }
    return phi;
}

// Which (i-block, split) a workgroup of a launch takes.  The hardware deals
// consecutive workgroups (x fastest) to the NXCD XCDs in turn, and each XCD
// has an L2 of its own: taken as (blockIdx.x, blockIdx.y), the i-blocks that
// run side by side on one XCD belong to several splits, and every XCD
// fetches every split's source records from memory.  Renumbered so that XCD
// k takes the k-th contiguous run of the pairs in x-fastest order, the
// workgroups resident on one XCD walk the same split's tiles together and
// share them in its L2.  A bijection of the grid for any size: the first
// (total mod NXCD) XCDs get one pair more.
__device__ __forceinline__ void xcd_order(int64_t &g, int &b)
{
    constexpr uint64_t NXCD = 8;
    const uint64_t nx = gridDim.x, tot = nx * gridDim.y;
    const uint64_t id = blockIdx.x + (uint64_t)blockIdx.y * nx;
    const uint64_t x = id % NXCD, r = id / NXCD, q = tot / NXCD, rem = tot % NXCD;
    const uint64_t l = x < rem ? x * (q + 1) + r : rem * (q + 1) + (x - rem) * q + r;
    g = (int64_t)(l % nx);
    b = (int)(l / nx);
}

// PHI: also sum the potential (nbody_force, the start-up pass); a block
// step's evaluation does not need it (the energy has its own pass).  IPT:
// active particles per lane group.
template <int PREC, int LPI, int NW, bool EPS0, bool PHI, int IPT>
__global__ __launch_bounds__(NW * 64) void force_kernel(
    typename Smem<PREC>::R J, ForceWork w, ForceOut out, double *part,
    int64_t n_act_total, double eps2)
{
    int64_t g;
    int b;
    xcd_order(g, b);
    force_block<PREC, LPI, NW, EPS0, PHI, IPT>(J, w, out, part, n_act_total, eps2, g, b);
}

// Potential energy of the stored state (paper Sect. 5.1): every unordered
// pair of a cluster once, FP64.  Particle i (local index l in a cluster of
// size n_c) takes the sources l + 1 .. l + W_l taken cyclically, with
// W_l = (n_c - 1) / 2 for odd n_c and, for even n_c, n_c / 2 for l < n_c / 2
// and n_c / 2 - 1 otherwise: each pair at cyclic distance d < n_c / 2 is
// then taken by exactly one of its ends, and the pair at d = n_c / 2 by the
// end with the smaller index, so sum_l W_l = n_c (n_c - 1) / 2 and every
// workgroup does the same work (no triangle).  A workgroup holds IB = 256
// consecutive particles, one per lane; the union of their windows (virtual
// positions ib0 + 1 .. last + W, folded back into the cluster) goes through
// LDS in tiles of 256, split over grid.y = B; lanes mask only the tiles at
// the two ends of the union.  Output: partial sums -sum m_j / r_ij per
// particle and split, out[b * bstride + i].
template <bool EPS0>
__global__ __launch_bounds__(256) void energy_kernel(const double *X, const double *Y,
                                                     const double *Z, const double *M,
                                                     ForceWork w, double *out, int64_t bstride,
                                                     double eps2)
{
    constexpr int NT = 256;
    __shared__ double s_x[NT], s_y[NT], s_z[NT], s_m[NT];
    const int64_t g = blockIdx.x;
    const int b = blockIdx.y;
    int c = 0;
    int64_t gfirst = 0;
    if (w.blk_cluster) {
        c = w.blk_cluster[g];
        if (c < 0)
            return;  // grid padding past the last i-block
        gfirst = w.blk_first[c];
    }
    const int64_t o0 = w.off[c];
    const int64_t nc = w.off[c + 1] - o0;
    const int64_t ib0 = (g - gfirst) * NT;          // local index of lane 0's particle
    const int64_t last = (ib0 + NT < nc ? ib0 + NT : nc) - 1;
    const int tid = threadIdx.x;
    const int64_t l = ib0 + tid;
    const bool valid = l < nc;
    const int64_t half = nc / 2;
    const int64_t wl = (nc & 1) ? half : (l < half ? half : half - 1);
    const int64_t wmin = (nc & 1) ? half : half - 1;   // smallest window of the cluster
    const int64_t i = o0 + (valid ? l : ib0);
    const double xi = X[i], yi = Y[i], zi = Z[i];

    // this split's share of the union of the windows, in whole tiles
    const int64_t u_beg = ib0 + 1, u_end = last + half + 1;
    int64_t chunk = (u_end - u_beg + w.split - 1) / w.split;
    chunk = (chunk + NT - 1) / NT * NT;
    const int64_t u0 = u_beg + (int64_t)b * chunk;
    const int64_t u1 = u0 + chunk < u_end ? u0 + chunk : u_end;

    double phi = 0.0;
    for (int64_t t0 = u0; t0 < u1; t0 += NT) {
        __syncthreads();
        const int64_t u = t0 + tid;
        if (u < u1) {
            const int64_t j = o0 + (u < nc ? u : u - nc);   // u < 2 n_c always
            s_x[tid] = X[j];
            s_y[tid] = Y[j];
            s_z[tid] = Z[j];
            s_m[tid] = M[j];
        } else {
            s_x[tid] = NULL_POS;
            s_y[tid] = NULL_POS;
            s_z[tid] = NULL_POS;
            s_m[tid] = 0.0;
        }
        __syncthreads();
        // slots s of this tile with 1 <= t0 + s - l <= w_l; every lane's
        // range covers the whole tile when t0 > last and t0 + NT - 1 <= ib0 + wmin
        if (t0 > last && t0 + NT - 1 <= ib0 + wmin) {
            phi = pot_tile<NT, false, EPS0>(s_x, s_y, s_z, s_m, xi, yi, zi, eps2, 0, NT - 1, phi);
        } else {
            const int64_t lo = l + 1 - t0, hi = l + wl - t0;
            const int slo = lo < 0 ? 0 : (lo > NT ? NT : (int)lo);
            const int shi = hi < -1 ? -1 : (hi > NT - 1 ? NT - 1 : (int)hi);
            phi = pot_tile<NT, true, EPS0>(s_x, s_y, s_z, s_m, xi, yi, zi, eps2, slo, shi, phi);
        }
    }
    if (valid)
        out[(int64_t)b * bstride + i] = phi;
}

// Sum the B split-source partials of every active slot in the fixed order
// b = 0 .. B-1 (Table 1, section 4 of the paper).  One thread per (quantity,
// active slot), so reads are coalesced over slots; the loads of 16 splits
// are issued before their adds (the order of the adds is unchanged), which
// keeps a tiny active set with a large B from waiting out B serial
// round trips to L2.  With the evaluation's ForceWork (w.off != nullptr),
// only the splits that hold sources of the slot's cluster are read (the
// evaluation's chunks are whole tiles of nt sources).
__global__ __launch_bounds__(256) void reduce_split(const double *part, int32_t B,
                                                    int64_t n_act, ForceOut out,
                                                    int pot_only, ForceWork w,
                                                    const int32_t *cluster_of, int nt)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int nq = pot_only ? 1 : 10;
    if (t >= n_act * nq)
        return;
    const int q = pot_only ? 9 : (int)(t / n_act);
    const int64_t k = pot_only ? t : t - (int64_t)q * n_act;
    const double *p = part + (int64_t)q * n_act + k;
    if (w.off) {
        const int64_t i = w.idx ? (int64_t)w.idx[k] : k;
        // (an index out of range was skipped by the evaluation: any cluster)
        const int c = cluster_of && i >= 0 && i < w.off[w.nc] ? cluster_of[i] : 0;
        B = (int32_t)splits_used(w.off[c + 1] - w.off[c], B, nt);
    }
    const int64_t stride = 10 * n_act;
    constexpr int U = 16;
    double r = 0.0;
    int b = 0;
    for (; b + U <= B; b += U) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            v[u] = p[(int64_t)(b + u) * stride];
#pragma unroll
        for (int u = 0; u < U; ++u)
            r += v[u];
    }
    for (; b < B; ++b)
        r += p[(int64_t)b * stride];
    if (q == 9) {
        if (out.pot)
            out.pot[k] = r;
    } else {
        out.vec[q / 3][k * out.sk + (q % 3) * out.sd] = r;
    }
}

// ---- dispatch table over the template parameters
using KMixed = void (*)(JRecMixed, ForceWork, ForceOut, double *, int64_t, double);
using KPair32 = void (*)(JRecPair32, ForceWork, ForceOut, double *, int64_t, double);
using KF64 = void (*)(JRecF64, ForceWork, ForceOut, double *, int64_t, double);

// Two active particles per lane group are built for 1, 2 and 4 lanes per
// particle (the large active sets, where the LDS reads per pair matter);
// smaller sets use one.
template <int PREC, bool EPS0, int NW, bool PHI>
auto pick_lpi(int lpi_log2, int ipt)
{
    using K = void (*)(typename Smem<PREC>::R, ForceWork, ForceOut, double *, int64_t, double);
    static const K tab[7] = {
        force_kernel<PREC, 1, NW, EPS0, PHI, 1>,  force_kernel<PREC, 2, NW, EPS0, PHI, 1>,
        force_kernel<PREC, 4, NW, EPS0, PHI, 1>,  force_kernel<PREC, 8, NW, EPS0, PHI, 1>,
        force_kernel<PREC, 16, NW, EPS0, PHI, 1>, force_kernel<PREC, 32, NW, EPS0, PHI, 1>,
        force_kernel<PREC, 64, NW, EPS0, PHI, 1>};
    static const K tab2[3] = {force_kernel<PREC, 1, NW, EPS0, PHI, 2>,
                              force_kernel<PREC, 2, NW, EPS0, PHI, 2>,
                              force_kernel<PREC, 4, NW, EPS0, PHI, 2>};
    return ipt == 2 && lpi_log2 <= 2 ? tab2[lpi_log2] : tab[lpi_log2];
}

template <int PREC, bool EPS0, bool PHI = true>
auto pick_kernel(int lpi_log2, int nw, int ipt = 1)
{
    if (nw == 1)
        return pick_lpi<PREC, EPS0, 1, PHI>(lpi_log2, ipt);
    if (nw == 2)
        return pick_lpi<PREC, EPS0, 2, PHI>(lpi_log2, ipt);
    return pick_lpi<PREC, EPS0, 4, PHI>(lpi_log2, ipt);
}

// the four (eps = 0, potential) variants of one precision
template <int PREC>
auto pick_variant(int lpi_log2, int nw, int ipt, bool eps0, bool phi)
{
    if (eps0)
        return phi ? pick_kernel<PREC, true, true>(lpi_log2, nw, ipt)
                   : pick_kernel<PREC, true, false>(lpi_log2, nw, ipt);
    return phi ? pick_kernel<PREC, false, true>(lpi_log2, nw, ipt)
               : pick_kernel<PREC, false, false>(lpi_log2, nw, ipt);
}

int ilog2(int64_t v)
{
    int r = 0;
    while ((int64_t(1) << (r + 1)) <= v)
        ++r;
    return r;
}

}  // namespace

int64_t iblock_size(const Launch &L) { return (int64_t)L.waves * (64 / L.lpi) * L.ipt; }

// Launch shape: the pinned one, else the autotuner's for this power of two
// of N_act, else a rule (below).
Launch pick_launch(const Ctx &c, int64_t n_act, int64_t n_src)
{
    if (c.pinned.lpi > 0)
        return c.pinned;
    if (n_act >= 1 && !c.tuned.empty()) {
        const int b = ilog2(n_act);
        if (b < (int)c.tuned.size() && c.tuned[b].lpi > 0) {
            Launch L = c.tuned[b];
            // at least one tile per split of the largest source range, and
            // the partials within the split buffer
            while (L.split > 1 && ((int64_t)L.split * n_act > c.part_cap ||
                                   n_src / L.split < 64 * L.waves))
                L.split >>= 1;
            return L;
        }
    }
    return rule_launch(n_act, n_src, c.part_cap, c.cfg.precision);
}

// Rule fitted to the autotuner's choices on 16,384- and 65,536-source
// spheres: 4 waves; about 4096 lanes per split (lanes per particle
// 4096 / N_act, between 1 and 64); two particles per lane group for active
// sets of 2^15 and more in the modes with FP64 pair arithmetic (it halves
// the LDS reads per pair: 1-3 % faster there, measured; the FP32-pair mode
// is faster with one); then split the sources while every split keeps two
// tiles, the partials (split x N_act slots) fit part_cap, and either the
// grid stays within 2^19 lanes or every split still holds 2^17 sources or
// more.  The second clause is for large source sets: there a split's work
// dwarfs its partials' traffic, and a grid of many more workgroups than the
// chip holds at once (3 per CU at the mixed kernel's register use) leaves
// a shorter partly empty last round.  Measured at 65,536 active x 8,388,608
// sources: split 16 / 32 / 64 / 128 / 256 -> 946 / 935 / 930 / 927 / 925 ms,
// but 3.4 / 4.5 / 6.8 / 11.2 / 20.2 GB fetched (shorter walks, started at
// staggered times, share the L2 less); 2^17 stops at 64.  For the same
// reason a grid of at most 4096 workgroups (about five rounds of the 768
// resident ones) is split further while every split keeps 2^15 sources:
// 131,072 active x 2^20 sources 241 -> 238 ms (split 8 -> 16), 65,536 x 2^21
// 243 -> 240 ms (16 -> 32), measured.
Launch rule_launch(int64_t n_act, int64_t n_src, int64_t part_cap, int prec)
{
    Launch L;
    L.waves = 4;
    L.lpi = 1;
    L.split = 1;
    while (n_act * L.lpi < 4096 && L.lpi < 64)
        L.lpi <<= 1;
    L.ipt = prec != NBODY_PREC_FP32PAIR && L.lpi <= 4 && n_act * L.lpi >= (int64_t(1) << 15) ? 2 : 1;
    const int64_t nt = 64 * L.waves;
    const int64_t max_lanes = int64_t(1) << 19, long_split = int64_t(1) << 17;
    const int64_t few_wgs = 4096, mid_split = int64_t(1) << 15;
    const int64_t n_ib = (n_act + iblock_size(L) - 1) / iblock_size(L);
    for (;;) {
        const int64_t b2 = (int64_t)L.split * 2, per_split = n_src / b2;
        if (per_split < 2 * nt || b2 * n_act > part_cap || b2 > 65535)   // grid y limit
            break;
        const bool lanes_ok = n_act * L.lpi / L.ipt * b2 <= max_lanes;
        const bool few = n_ib * b2 <= few_wgs && per_split >= mid_split;
        if (!lanes_ok && per_split < long_split && !few)
            break;
        L.split <<= 1;
    }
    return L;
}

hipError_t launch_force(Ctx &c, const ForceWork &w, const Launch &L,
                        const ForceOut &out, int64_t n_act_total, hipStream_t s, bool reduce)
{
    if (n_act_total <= 0 || w.n_blocks <= 0)
        return hipSuccess;
    const int lg = ilog2(L.lpi);
    const bool eps0 = c.eps == 0.0;
    const double eps2 = c.eps * c.eps;
    double *part = w.split > 1 ? c.part : nullptr;
    const dim3 grid((unsigned)w.n_blocks, (unsigned)w.split);
    const dim3 block(64 * L.waves);
    const int prec = c.cfg.precision;
    const bool phi = out.pot != nullptr;   // potential wanted (not in block steps)
    const int rec = prof_begin(c, PH_FORCE, n_act_total);
    if (prec == NBODY_PREC_MIXED) {
        const KMixed k = pick_variant<PREC_MIXED>(lg, L.waves, L.ipt, eps0, phi);
        hipLaunchKernelGGL(k, grid, block, 0, s, c.jm, w, out, part, n_act_total, eps2);
    } else if (prec == NBODY_PREC_FP32PAIR) {
        const KPair32 k = pick_variant<PREC_PAIR32>(lg, L.waves, L.ipt, eps0, phi);
        hipLaunchKernelGGL(k, grid, block, 0, s, c.jp, w, out, part, n_act_total, eps2);
    } else {
        const KF64 k = pick_variant<PREC_F64>(lg, L.waves, L.ipt, eps0, phi);
        hipLaunchKernelGGL(k, grid, block, 0, s, c.jd, w, out, part, n_act_total, eps2);
    }
    prof_end(c, rec);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || w.split <= 1 || !reduce)
        return e;
    const unsigned nb = (unsigned)((n_act_total * 10 + 255) / 256);
    const int rr = prof_begin(c, PH_REDUCE);
    hipLaunchKernelGGL(reduce_split, dim3(nb), dim3(256), 0, s, (const double *)c.part,
                       w.split, n_act_total, out, 0, w, (const int32_t *)c.d_cluster_of,
                       64 * L.waves);
    prof_end(c, rr);
    return hipGetLastError();
}

// Potential of the stored state for the energy: phi[i] = -sum over the
// particle's half-window of m_j / r_ij (every pair of a cluster once).
hipError_t launch_energy_pot(Ctx &c, double *phi, hipStream_t s)
{
    constexpr int64_t IB = 256;
    const int64_t n = c.n;
    hipError_t e = launch_segments(c, nullptr, n, s);
    if (e != hipSuccess)
        return e;
    ForceWork w{};
    w.seg = c.d_seg;
    w.off = c.d_off;
    w.nc = c.nc;
    if (c.nc == 1) {
        w.n_blocks = (n + IB - 1) / IB;
    } else {
        const int64_t cap = n / IB + c.nc + 1;
        if ((e = launch_blocks(c, IB, cap, s)) != hipSuccess)
            return e;
        w.blk_cluster = c.d_blk_cluster;
        w.blk_first = c.d_blk_first;
        w.n_blocks = cap;
    }
    // splits: up to ~2048 workgroups, at least two tiles per split, and the
    // partial sums within the split buffer
    int64_t ncmax = 0;
    for (size_t k = 0; k + 1 < c.off.size(); ++k)
        ncmax = std::max(ncmax, c.off[k + 1] - c.off[k]);
    int split = 1;
    while (w.n_blocks * split * 2 <= 2048 && (ncmax / 2 + IB) / (split * 2) >= 2 * IB &&
           (int64_t)split * 2 * n <= c.part_cap)
        split <<= 1;
    w.split = split;
    const double *X = c.st.pos, *Y = c.st.pos + n, *Z = c.st.pos + 2 * n;
    double *dst = split > 1 ? c.part + 9 * n : phi;
    const int64_t bstride = 10 * n;   // the [B][10][n] layout of the split buffer, slot 9
    auto k = c.eps == 0.0 ? energy_kernel<true> : energy_kernel<false>;
    const int rec = prof_begin(c, PH_ENERGY);
    hipLaunchKernelGGL(k, dim3((unsigned)w.n_blocks, (unsigned)split), dim3(IB), 0, s, X, Y, Z,
                       (const double *)c.st.mass, w, dst, bstride, c.eps * c.eps);
    if ((e = hipGetLastError()) != hipSuccess || split == 1) {
        prof_end(c, rec);
        return e;
    }
    ForceOut out{};
    out.pot = phi;
    hipLaunchKernelGGL(reduce_split, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       (const double *)c.part, split, n, out, 1, ForceWork{},
                       (const int32_t *)nullptr, 0);
    prof_end(c, rec);
    return hipGetLastError();
}

hipError_t launch_force_init(Ctx &c, const ForceWork &w, const Launch &L,
                             const ForceOut &out, hipStream_t s)
{
    if (w.n_blocks <= 0)
        return hipSuccess;
    JRecF64 J{};
    J.x = c.st.pos; J.y = c.st.pos + c.n; J.z = c.st.pos + 2 * c.n;
    J.vx = c.st.vel; J.vy = c.st.vel + c.n; J.vz = c.st.vel + 2 * c.n;
    J.ax = c.st.acc; J.ay = c.st.acc + c.n; J.az = c.st.acc + 2 * c.n;
    J.jx = c.st.jrk; J.jy = c.st.jrk + c.n; J.jz = c.st.jrk + 2 * c.n;
    J.m = c.st.mass;
    ForceWork w1 = w;
    w1.split = 1;
    const int lg = ilog2(L.lpi);
    KF64 k = c.eps == 0.0 ? pick_kernel<PREC_INIT, true>(lg, L.waves)
                          : pick_kernel<PREC_INIT, false>(lg, L.waves);
    hipLaunchKernelGGL(k, dim3((unsigned)w1.n_blocks, 1), dim3(64 * L.waves), 0, s, J, w1, out,
                       (double *)nullptr, (int64_t)0, c.eps * c.eps);
    return hipGetLastError();
}

}  // namespace nb
