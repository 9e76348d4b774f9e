// Evaluation step of the Hermite scheme (paper Sect. 3, item 2, with the
// softened potential of Sect. 2): the per-workgroup body shared by the
// launch kernel (force.hip) and the device-resident block-step loop
// (integrate.hip).  The design notes are at the top of force.hip.
#pragma once
#include "nbody_internal.h"

namespace nb {

namespace {

// kernel variants: the two public mixed modes, the FP64 path and the
// start-up pass
constexpr int PREC_MIXED = 0, PREC_F64 = 1, PREC_INIT = 3, PREC_PAIR32 = 4;

// Knuth's two-sum: (hi, lo) += p without rounding loss in the (hi, lo) pair.
__device__ __forceinline__ void ds_add(float &hi, float &lo, float p)
{
    const float s = hi + p;
    const float bp = s - hi;
    const float e = (hi - (s - bp)) + (p - bp);
    hi = s;
    lo += e;
}

// Far-away, massless stand-in for source slots past the end of a range.
constexpr double NULL_POS = 1.0e15;

template <int PREC>
struct Smem;

template <>
struct Smem<PREC_MIXED> {
    using R = JRecMixed;
};
template <>
struct Smem<PREC_PAIR32> {
    using R = JRecPair32;
};
template <>
struct Smem<PREC_F64> {
    using R = JRecF64;
};
template <>
struct Smem<PREC_INIT> {
    using R = JRecF64;
};

// 1/sqrt(r2) for the mixed path: FP32 seed from v_rsq_f32 (|error| < 1 ulp,
// measured) and one Newton step in FP64, which squares the relative error
// (~1e-14).  Used for the acceleration and potential terms and, with the
// same operations, for the removal of the j == i potential term.
__device__ __forceinline__ double rinv_mixed(double r2)
{
    const double y0 = (double)__builtin_amdgcn_rsqf((float)r2);
    const double res = fma(-r2 * y0, y0, 1.0);   // 1 - r2 y0^2
    return fma(0.5 * y0, res, y0);
}

// 1/sqrt(r2) to FP64 accuracy for the FP64 passes: the same FP32 seed y0
// (relative error |d| below ~2e-7 with the rounding of r2 to FP32), then the
// third-order step y0 (1 + e/2 + 3e^2/8), e = 1 - r2 y0^2 = O(2d), whose
// truncation error (5/16) e^3 is far below an FP64 ulp; the result is within
// about one ulp.  Valid while r2 is a normal FP32 number (r from ~1e-19 to
// ~1e19), which the softened distances of every supported system are.
__device__ __forceinline__ double rinv_f64(double r2)
{
    const double y0 = (double)__builtin_amdgcn_rsqf((float)r2);
    const double e = fma(-r2 * y0, y0, 1.0);
    return fma(y0 * e, fma(e, 0.375, 0.5), y0);
}

// LDS tile of NT source records, one 16-byte aligned record per source
// (its fields side by side): with one lane per particle every lane reads
// the same record, and from one address every field is an immediate offset
// (with one array per field the compiler formed each field's address apart
// and copied it into a vector register per read: 2-5 % more VALU
// instructions per pair).  One tile per (precision, tile size): every
// launch shape with that tile size uses the same LDS, so a kernel that runs
// several shapes (the ensemble loop) holds one tile.
template <int PREC, int NT>
struct SrcTile {
    static constexpr bool P32 = PREC == PREC_PAIR32, MIXED = PREC == PREC_MIXED;
    static constexpr int NJ = PREC == PREC_INIT ? NT : 1;
    using VV = typename std::conditional<P32, float, double>::type;
    using VA = typename std::conditional<MIXED || P32, float, double>::type;
    struct alignas(16) S {
        double x, y, z, m;
        VV vx, vy, vz;
        VA ax, ay, az;
    };
    S s[NT];
    double jx[NJ], jy[NJ], jz[NJ];   // sources' jerks: start-up evaluation only
};

template <int PREC, int NT>
__device__ __forceinline__ SrcTile<PREC, NT> &src_tile()
{
    __shared__ SrcTile<PREC, NT> t;
    return t;
}

// One workgroup's share of an evaluation: i-block g (IB active slots) against
// source split b.  The launch kernel calls it with (blockIdx.x, blockIdx.y);
// the device-resident block-step loop calls it for the units it takes.
// Every early return is uniform over the workgroup.  PHI: also sum the
// potential (nbody_force, the start-up pass); a block step's evaluation
// does not need it (the energy has its own pass).  IPT: active particles
// per lane group (each source read from LDS serves IPT pairs).
template <int PREC, int LPI, int NW, bool EPS0, bool PHI, int IPT = 1>
__device__ __forceinline__ void force_block(const typename Smem<PREC>::R &J, const ForceWork &w,
                                            const ForceOut &out, double *part,
                                            int64_t n_act_total, double eps2, int64_t g,
                                            int b)
{
    constexpr int NT = NW * 64;      // sources per LDS tile
    constexpr int GI = 64 / LPI;     // lane groups (of LPI lanes) per wave
    constexpr int NG = NW * GI;      // lane groups per workgroup
    constexpr int IB = NG * IPT;     // active particles per workgroup
    constexpr int PER = NT / LPI;    // sources per lane per tile
    constexpr bool MIXED = PREC == PREC_MIXED;
    constexpr bool P32 = PREC == PREC_PAIR32;
    constexpr bool INIT = PREC == PREC_INIT;
    constexpr int NV = INIT ? 12 : 9;   // vector outputs (3 components each)
    // FP32 accumulators (mixed: snap; FP32-pair mode: all nine); FP64 ones
    // for the rest
    constexpr int NF = MIXED ? 3 : (P32 ? 9 : 1);
    constexpr int ND = MIXED ? 6 : (P32 ? 1 : NV);
    // types of the sources' velocity and acceleration (as in the records)
    using VV = typename std::conditional<P32, float, double>::type;
    using VA = typename std::conditional<MIXED || P32, float, double>::type;

    SrcTile<PREC, NT> &tl = src_tile<PREC, NT>();

    // ---- which active slots and which sources this workgroup takes
    int c = 0;
    int64_t gfirst = 0;
    if (w.blk_cluster) {
        c = w.blk_cluster[g];
        if (c < 0)
            return;  // grid padding past the last i-block
        gfirst = w.blk_first[c];
    }
    const int64_t s0 = w.seg[c], s1 = w.seg[c + 1];
    const int64_t kb = s0 + (g - gfirst) * IB;
    const int64_t o0 = w.off[c], o1 = w.off[c + 1];
    const int64_t chunk = split_chunk(o1 - o0, w.split, NT);
    // splits past this cluster's sources (chunks are whole tiles, so a small
    // cluster fills fewer than B of them): nothing to do, and the reduction
    // reads only the splits in use
    if ((int64_t)b * chunk >= o1 - o0 && b > 0)
        return;
    const int64_t j0 = o0 + (int64_t)b * chunk;
    const int64_t j1 = j0 + chunk < o1 ? j0 + chunk : o1;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int il = wave * GI + lane / LPI;   // lane group
    const int js = lane & (LPI - 1);         // slot within the group
    // particle u of the lane group: active slot kb + il + u NG
    int64_t k[IPT], i[IPT];
    bool valid[IPT];
    double xi[IPT], yi[IPT], zi[IPT];
    VV vxi[IPT], vyi[IPT], vzi[IPT];
    VA axi[IPT], ayi[IPT], azi[IPT];
    double jxi[IPT], jyi[IPT], jzi[IPT];
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
        k[u] = kb + il + u * NG;
        valid[u] = k[u] < s1;
        const int64_t kk = valid[u] ? k[u] : kb;
        i[u] = w.idx ? (int64_t)w.idx[kk] : kk;
        if (i[u] < o0 || i[u] >= o1) {
            // an index outside its cluster (a caller's bad list): skip the
            // slot, load a valid particle, report
            if (valid[u] && js == 0 && w.err)
                atomicOr(w.err, ERR_BADIDX);
            valid[u] = false;
            i[u] = o0;
        }
        xi[u] = J.x[i[u]]; yi[u] = J.y[i[u]]; zi[u] = J.z[i[u]];
        vxi[u] = J.vx[i[u]]; vyi[u] = J.vy[i[u]]; vzi[u] = J.vz[i[u]];
        axi[u] = J.ax[i[u]]; ayi[u] = J.ay[i[u]]; azi[u] = J.az[i[u]];
        jxi[u] = 0; jyi[u] = 0; jzi[u] = 0;
        if constexpr (INIT) {
            jxi[u] = J.jx[i[u]]; jyi[u] = J.jy[i[u]]; jzi[u] = J.jz[i[u]];
        }
    }

    // FP64 sums (mixed: acceleration and jerk; FP64 passes: everything),
    // the potential in FP64 always, and double-single (hi, lo) pairs for
    // the FP32 sums (mixed: snap; FP32-pair mode: everything), fed by FP32
    // partial sums over at most FOLD pairs per lane
    double D[IPT][ND];
    float H[IPT][NF], L[IPT][NF];
    double phi[IPT];
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
#pragma unroll
        for (int q = 0; q < ND; ++q)
            D[u][q] = 0.0;
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            H[u][q] = 0.0f;
            L[u][q] = 0.0f;
        }
        phi[u] = 0.0;
    }

    for (int64_t t0 = j0; t0 < j1; t0 += NT) {
        __syncthreads();
        const int64_t jj = t0 + tid;
        if (jj < j1) {
            tl.s[tid].x = J.x[jj];
            tl.s[tid].y = J.y[jj];
            tl.s[tid].z = J.z[jj];
            tl.s[tid].m = J.m[jj];
            tl.s[tid].vx = J.vx[jj]; tl.s[tid].vy = J.vy[jj]; tl.s[tid].vz = J.vz[jj];
            tl.s[tid].ax = J.ax[jj]; tl.s[tid].ay = J.ay[jj]; tl.s[tid].az = J.az[jj];
            if constexpr (INIT) {
                tl.jx[tid] = J.jx[jj]; tl.jy[tid] = J.jy[jj]; tl.jz[tid] = J.jz[jj];
            }
        } else {
            tl.s[tid].x = NULL_POS;
            tl.s[tid].y = NULL_POS;
            tl.s[tid].z = NULL_POS;
            tl.s[tid].m = 0.0;
            tl.s[tid].vx = 0; tl.s[tid].vy = 0; tl.s[tid].vz = 0;
            tl.s[tid].ax = 0; tl.s[tid].ay = 0; tl.s[tid].az = 0;
            if constexpr (INIT) {
                tl.jx[tid] = 0; tl.jy[tid] = 0; tl.jz[tid] = 0;
            }
        }
        __syncthreads();

        // a short FP32 partial keeps its rounding small (64 pairs measured
        // 3x better than 256 for FP32 jerk sums, at ~1% more instructions)
        constexpr int FOLD = (MIXED || P32) ? (PER < 64 ? PER : 64) : PER;
        for (int p0 = 0; p0 < PER; p0 += FOLD) {
            float T[IPT][NF];
#pragma unroll
            for (int u = 0; u < IPT; ++u)
#pragma unroll
                for (int q = 0; q < NF; ++q)
                    T[u][q] = 0.0f;

            constexpr int UNROLL = IPT == 1 ? 4 : 2;
#pragma unroll UNROLL
            for (int p = p0; p < p0 + FOLD; ++p) {
                const int t = js + p * LPI;
                const auto &sr = tl.s[t];
                const double sx = sr.x, sy = sr.y, sz = sr.z, sm = sr.m;
                const VV svx = sr.vx, svy = sr.vy, svz = sr.vz;
                const VA sax = sr.ax, say = sr.ay, saz = sr.az;
#pragma unroll
                for (int u = 0; u < IPT; ++u) {
                    if constexpr (P32) {
                        // every pair term in FP32 from the FP64 difference r_j - r_i
                        const float dx = (float)(sx - xi[u]), dy = (float)(sy - yi[u]),
                                    dz = (float)(sz - zi[u]);
                        const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, (float)eps2)));
                        float rinv = __builtin_amdgcn_rsqf(r2);
                        if constexpr (EPS0)
                            rinv = r2 > 0.0f ? rinv : 0.0f;
                        const float mrinv = (float)sm * rinv;
                        if constexpr (PHI)
                            phi[u] -= (double)mrinv;
                        const float rinv2 = rinv * rinv, mr3 = mrinv * rinv2;
                        const float dvx = svx - vxi[u], dvy = svy - vyi[u], dvz = svz - vzi[u];
                        const float dax = sax - axi[u], day = say - ayi[u], daz = saz - azi[u];
                        const float rv = fmaf(dx, dvx, fmaf(dy, dvy, dz * dvz));
                        const float qq = fmaf(dvx, dvx, fmaf(dvy, dvy, fmaf(dvz, dvz,
                                         fmaf(dx, dax, fmaf(dy, day, dz * daz)))));
                        const float alpha = rv * rinv2;
                        const float beta = fmaf(alpha, alpha, qq * rinv2);
                        const float a3 = -3.0f * alpha, a6 = a3 + a3, b3 = -3.0f * beta;
                        const float jx = fmaf(a3, dx, dvx), jy = fmaf(a3, dy, dvy),
                                    jz = fmaf(a3, dz, dvz);
                        float *Tu = T[u];
                        Tu[0] = fmaf(mr3, dx, Tu[0]);
                        Tu[1] = fmaf(mr3, dy, Tu[1]);
                        Tu[2] = fmaf(mr3, dz, Tu[2]);
                        Tu[3] = fmaf(mr3, jx, Tu[3]);
                        Tu[4] = fmaf(mr3, jy, Tu[4]);
                        Tu[5] = fmaf(mr3, jz, Tu[5]);
                        Tu[6] = fmaf(mr3, fmaf(a6, jx, fmaf(b3, dx, dax)), Tu[6]);
                        Tu[7] = fmaf(mr3, fmaf(a6, jy, fmaf(b3, dy, day)), Tu[7]);
                        Tu[8] = fmaf(mr3, fmaf(a6, jz, fmaf(b3, dz, daz)), Tu[8]);
                        continue;
                    }
                    const double dxd = sx - xi[u], dyd = sy - yi[u], dzd = sz - zi[u];
                    const double r2 = fma(dxd, dxd, fma(dyd, dyd, fma(dzd, dzd, eps2)));
                    double rinv;
                    if constexpr (MIXED)
                        rinv = rinv_mixed(r2);
                    else
                        rinv = rinv_f64(r2);
                    if constexpr (EPS0)
                        rinv = r2 > 0.0 ? rinv : 0.0;
                    const double mrinv = sm * rinv;
                    if constexpr (PHI)
                        phi[u] -= mrinv;
                    const double rinv2 = rinv * rinv;
                    const double mr3 = mrinv * rinv2;
                    double *Du = D[u];
                    if constexpr (MIXED) {
                        // acceleration and jerk in FP64, snap in FP32:
                        // A = m r^-3 r, J = m r^-3 (v - 3 alpha r),
                        // S = m r^-3 (a - 6 alpha jv - 3 beta r), jv = v - 3 alpha r
                        Du[0] = fma(mr3, dxd, Du[0]);
                        Du[1] = fma(mr3, dyd, Du[1]);
                        Du[2] = fma(mr3, dzd, Du[2]);
                        const double dvx = svx - vxi[u], dvy = svy - vyi[u], dvz = svz - vzi[u];
                        const double m3r2 = -3.0 * rinv2;
                        const double a3d = fma(dxd, dvx, fma(dyd, dvy, dzd * dvz)) * m3r2;  // -3 alpha
                        const double jxd = fma(a3d, dxd, dvx), jyd = fma(a3d, dyd, dvy),
                                     jzd = fma(a3d, dzd, dvz);
                        Du[3] = fma(mr3, jxd, Du[3]);
                        Du[4] = fma(mr3, jyd, Du[4]);
                        Du[5] = fma(mr3, jzd, Du[5]);
                        const float dx = (float)dxd, dy = (float)dyd, dz = (float)dzd;
                        const float fvx = (float)dvx, fvy = (float)dvy, fvz = (float)dvz;
                        const float jx = (float)jxd, jy = (float)jyd, jz = (float)jzd;
                        const float a3 = (float)a3d, f3r2 = (float)m3r2, fm3 = (float)mr3;
                        const float dax = sax - axi[u], day = say - ayi[u], daz = saz - azi[u];
                        const float qq = fmaf(fvx, fvx, fmaf(fvy, fvy, fmaf(fvz, fvz,
                                         fmaf(dx, dax, fmaf(dy, day, dz * daz)))));
                        // -3 beta = -3 alpha^2 - 3 qq / s^2, with alpha = -a3 / 3
                        const float b3 = fmaf(a3, a3 * (-1.0f / 3.0f), qq * f3r2);
                        const float a6 = a3 + a3;
                        const float sxf = fmaf(a6, jx, fmaf(b3, dx, dax));
                        const float syf = fmaf(a6, jy, fmaf(b3, dy, day));
                        const float szf = fmaf(a6, jz, fmaf(b3, dz, daz));
                        T[u][0] = fmaf(fm3, sxf, T[u][0]);
                        T[u][1] = fmaf(fm3, syf, T[u][1]);
                        T[u][2] = fmaf(fm3, szf, T[u][2]);
                    } else {
                        const double dvx = svx - vxi[u], dvy = svy - vyi[u], dvz = svz - vzi[u];
                        const double dax = sax - axi[u], day = say - ayi[u], daz = saz - azi[u];
                        const double alpha = fma(dxd, dvx, fma(dyd, dvy, dzd * dvz)) * rinv2;
                        const double qq = fma(dvx, dvx, fma(dvy, dvy, fma(dvz, dvz,
                                          fma(dxd, dax, fma(dyd, day, dzd * daz)))));
                        const double beta = fma(alpha, alpha, qq * rinv2);
                        if constexpr (INIT) {
                            // start-up evaluation with the crackle, term by term
                            const double djx = tl.jx[t] - jxi[u], djy = tl.jy[t] - jyi[u],
                                         djz = tl.jz[t] - jzi[u];
                            const double gamma = (3.0 * (dvx * dax + dvy * day + dvz * daz) +
                                                  dxd * djx + dyd * djy + dzd * djz) * rinv2 +
                                                 alpha * (3.0 * beta - 4.0 * alpha * alpha);
                            const double Ax = mr3 * dxd, Ay = mr3 * dyd, Az = mr3 * dzd;
                            const double Jx = mr3 * dvx - 3.0 * alpha * Ax;
                            const double Jy = mr3 * dvy - 3.0 * alpha * Ay;
                            const double Jz = mr3 * dvz - 3.0 * alpha * Az;
                            const double Sx = mr3 * dax - 6.0 * alpha * Jx - 3.0 * beta * Ax;
                            const double Sy = mr3 * day - 6.0 * alpha * Jy - 3.0 * beta * Ay;
                            const double Sz = mr3 * daz - 6.0 * alpha * Jz - 3.0 * beta * Az;
                            Du[0] += Ax; Du[1] += Ay; Du[2] += Az;
                            Du[3] += Jx; Du[4] += Jy; Du[5] += Jz;
                            Du[6] += Sx; Du[7] += Sy; Du[8] += Sz;
                            Du[ND - 3] += mr3 * djx - 9.0 * alpha * Sx - 9.0 * beta * Jx - 3.0 * gamma * Ax;
                            Du[ND - 2] += mr3 * djy - 9.0 * alpha * Sy - 9.0 * beta * Jy - 3.0 * gamma * Ay;
                            Du[ND - 1] += mr3 * djz - 9.0 * alpha * Sz - 9.0 * beta * Jz - 3.0 * gamma * Az;
                        } else {
                            const double a3 = -3.0 * alpha, a6 = a3 + a3, b3 = -3.0 * beta;
                            const double jx = fma(a3, dxd, dvx), jy = fma(a3, dyd, dvy),
                                         jz = fma(a3, dzd, dvz);
                            Du[0] = fma(mr3, dxd, Du[0]);
                            Du[1] = fma(mr3, dyd, Du[1]);
                            Du[2] = fma(mr3, dzd, Du[2]);
                            Du[3] = fma(mr3, jx, Du[3]);
                            Du[4] = fma(mr3, jy, Du[4]);
                            Du[5] = fma(mr3, jz, Du[5]);
                            Du[6] = fma(mr3, fma(a6, jx, fma(b3, dxd, dax)), Du[6]);
                            Du[7] = fma(mr3, fma(a6, jy, fma(b3, dyd, day)), Du[7]);
                            Du[8] = fma(mr3, fma(a6, jz, fma(b3, dzd, daz)), Du[8]);
                        }
                    }
                }
            }
            if constexpr (MIXED || P32) {
#pragma unroll
                for (int u = 0; u < IPT; ++u)
#pragma unroll
                    for (int q = 0; q < NF; ++q)
                        ds_add(H[u][q], L[u][q], T[u][q]);
            }
        }
    }

#pragma unroll
    for (int u = 0; u < IPT; ++u) {
        // ---- combine the LPI lanes of each active particle (xor butterfly)
        double R[NV + 1];
        if constexpr (P32) {
#pragma unroll
            for (int q = 0; q < NF; ++q)
                R[q] = (double)H[u][q] + (double)L[u][q];
        } else if constexpr (MIXED) {
#pragma unroll
            for (int q = 0; q < 6; ++q)
                R[q] = D[u][q];
#pragma unroll
            for (int q = 0; q < NF; ++q)
                R[6 + q] = (double)H[u][q] + (double)L[u][q];
        } else {
#pragma unroll
            for (int q = 0; q < NV; ++q)
                R[q] = D[u][q];
        }
        R[NV] = phi[u];
#pragma unroll
        for (int msk = 1; msk < LPI; msk <<= 1) {
#pragma unroll
            for (int q = 0; q < NV + 1; ++q)
                R[q] += __shfl_xor(R[q], msk, 64);
        }

        if (!valid[u] || js != 0)
            continue;
        const int64_t ku = k[u], iu = i[u];
        // the j == i pair adds exactly zero to a, da, d2a but -m_i / eps to the
        // potential: remove that term, computed with the same operations
        if constexpr (!EPS0 && PHI) {
            if (iu >= j0 && iu < j1) {
                if constexpr (P32) {
                    const float e2f = (float)eps2;
                    const float ri = __builtin_amdgcn_rsqf(fmaf(0.0f, 0.0f, fmaf(0.0f, 0.0f, fmaf(0.0f, 0.0f, e2f))));
                    R[NV] += (double)((float)J.m[iu] * ri);
                } else {
                    const double r2 = fma(0.0, 0.0, fma(0.0, 0.0, fma(0.0, 0.0, eps2)));
                    const double ri = MIXED ? rinv_mixed(r2) : rinv_f64(r2);
                    R[NV] += J.m[iu] * ri;
                }
            }
        }
        if constexpr (INIT) {
#pragma unroll
            for (int q = 0; q < NV / 3; ++q)
                if (out.vec[q])
#pragma unroll
                    for (int d = 0; d < 3; ++d)
                        out.vec[q][ku * out.sk + d * out.sd] = R[3 * q + d];
            continue;
        }
        if (part) {
            double *pb = part + (int64_t)b * 10 * n_act_total + ku;
#pragma unroll
            for (int q = 0; q < 10; ++q)
                pb[(int64_t)q * n_act_total] = R[q];
        } else {
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    out.vec[q][ku * out.sk + d * out.sd] = R[3 * q + d];
            if (out.pot)
                out.pot[ku] = R[NV];
        }
    }
}

}  // namespace

}  // namespace nb
