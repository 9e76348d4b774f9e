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
    using R = JRecMixed;
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

// One workgroup's share of an evaluation: i-block g (IB active slots) against
// source split b.  The launch kernel calls it with (blockIdx.x, blockIdx.y);
// the device-resident block-step loop calls it for the units it takes.
// Every early return is uniform over the workgroup.  PHI: also sum the
// potential (nbody_force, the start-up pass); a block step's evaluation
// does not need it (the energy has its own pass).
template <int PREC, int LPI, int NW, bool EPS0, bool PHI>
__device__ __forceinline__ void force_block(const typename Smem<PREC>::R &J, const ForceWork &w,
                                            const ForceOut &out, double *part,
                                            int64_t n_act_total, double eps2, int64_t g,
                                            int b)
{
    constexpr int NT = NW * 64;      // sources per LDS tile
    constexpr int GI = 64 / LPI;     // active particles per wave
    constexpr int IB = NW * GI;      // active particles per workgroup
    constexpr int PER = NT / LPI;    // pairs per lane per tile
    constexpr bool MIXED = PREC == PREC_MIXED;
    constexpr bool P32 = PREC == PREC_PAIR32;
    constexpr bool INIT = PREC == PREC_INIT;
    constexpr int NV = INIT ? 12 : 9;   // vector outputs (3 components each)
    // FP32 accumulators (mixed: jerk and snap; FP32-pair mode: all nine);
    // FP64 ones for the rest
    constexpr int NF = MIXED ? 6 : (P32 ? 9 : 1);
    constexpr int ND = MIXED ? 3 : (P32 ? 1 : NV);
    using VT = typename std::conditional<MIXED || P32, float, double>::type;

    __shared__ double s_x[NT], s_y[NT], s_z[NT], s_m[NT];
    __shared__ VT s_vx[NT], s_vy[NT], s_vz[NT];
    __shared__ VT s_ax[NT], s_ay[NT], s_az[NT];
    __shared__ double s_jx[INIT ? NT : 1], s_jy[INIT ? NT : 1], s_jz[INIT ? NT : 1];

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
    const int il = wave * GI + lane / LPI;
    const int js = lane & (LPI - 1);
    const int64_t k = kb + il;
    const bool valid = k < s1;
    const int64_t kk = valid ? k : kb;
    const int64_t i = w.idx ? (int64_t)w.idx[kk] : kk;

    const double xi = J.x[i], yi = J.y[i], zi = J.z[i];
    const VT vxi = J.vx[i], vyi = J.vy[i], vzi = J.vz[i];
    const VT axi = J.ax[i], ayi = J.ay[i], azi = J.az[i];
    double jxi = 0, jyi = 0, jzi = 0;
    if constexpr (INIT) {
        jxi = J.jx[i]; jyi = J.jy[i]; jzi = J.jz[i];
    }

    // FP64 sums (mixed: acceleration; otherwise everything), the potential
    // in FP64 always, and double-single (hi, lo) pairs for the mixed jerk
    // and snap, fed by FP32 partial sums over at most FOLD pairs per lane
    double D[ND];
#pragma unroll
    for (int q = 0; q < ND; ++q)
        D[q] = 0.0;
    float H[NF], L[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        H[q] = 0.0f;
        L[q] = 0.0f;
    }
    double phi = 0.0;

    for (int64_t t0 = j0; t0 < j1; t0 += NT) {
        __syncthreads();
        const int64_t jj = t0 + tid;
        if (jj < j1) {
            s_x[tid] = J.x[jj];
            s_y[tid] = J.y[jj];
            s_z[tid] = J.z[jj];
            s_m[tid] = J.m[jj];
            s_vx[tid] = J.vx[jj]; s_vy[tid] = J.vy[jj]; s_vz[tid] = J.vz[jj];
            s_ax[tid] = J.ax[jj]; s_ay[tid] = J.ay[jj]; s_az[tid] = J.az[jj];
            if constexpr (INIT) {
                s_jx[tid] = J.jx[jj]; s_jy[tid] = J.jy[jj]; s_jz[tid] = J.jz[jj];
            }
        } else {
            s_x[tid] = NULL_POS;
            s_y[tid] = NULL_POS;
            s_z[tid] = NULL_POS;
            s_m[tid] = 0.0;
            s_vx[tid] = 0; s_vy[tid] = 0; s_vz[tid] = 0;
            s_ax[tid] = 0; s_ay[tid] = 0; s_az[tid] = 0;
            if constexpr (INIT) {
                s_jx[tid] = 0; s_jy[tid] = 0; s_jz[tid] = 0;
            }
        }
        __syncthreads();

        // a short FP32 partial keeps its rounding small (64 pairs measured
        // 3x better than 256 for the jerk, at ~1% more instructions)
        constexpr int FOLD = (MIXED || P32) ? (PER < 64 ? PER : 64) : PER;
        for (int p0 = 0; p0 < PER; p0 += FOLD) {
            float T[NF];
#pragma unroll
            for (int q = 0; q < NF; ++q)
                T[q] = 0.0f;

#pragma unroll 4
            for (int p = p0; p < p0 + FOLD; ++p) {
                const int t = js + p * LPI;
                if constexpr (P32) {
                    // every pair term in FP32 from the FP64 difference r_j - r_i
                    const float dx = (float)(s_x[t] - xi), dy = (float)(s_y[t] - yi),
                                dz = (float)(s_z[t] - zi);
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, (float)eps2)));
                    float rinv = __builtin_amdgcn_rsqf(r2);
                    if constexpr (EPS0)
                        rinv = r2 > 0.0f ? rinv : 0.0f;
                    const float mrinv = (float)s_m[t] * rinv;
                    if constexpr (PHI)
                        phi -= (double)mrinv;
                    const float rinv2 = rinv * rinv, mr3 = mrinv * rinv2;
                    const float dvx = s_vx[t] - vxi, dvy = s_vy[t] - vyi, dvz = s_vz[t] - vzi;
                    const float dax = s_ax[t] - axi, day = s_ay[t] - ayi, daz = s_az[t] - azi;
                    const float rv = fmaf(dx, dvx, fmaf(dy, dvy, dz * dvz));
                    const float qq = fmaf(dvx, dvx, fmaf(dvy, dvy, fmaf(dvz, dvz,
                                     fmaf(dx, dax, fmaf(dy, day, dz * daz)))));
                    const float alpha = rv * rinv2;
                    const float beta = fmaf(alpha, alpha, qq * rinv2);
                    const float a3 = -3.0f * alpha, a6 = a3 + a3, b3 = -3.0f * beta;
                    const float jx = fmaf(a3, dx, dvx), jy = fmaf(a3, dy, dvy), jz = fmaf(a3, dz, dvz);
                    T[0] = fmaf(mr3, dx, T[0]);
                    T[1] = fmaf(mr3, dy, T[1]);
                    T[2] = fmaf(mr3, dz, T[2]);
                    T[3] = fmaf(mr3, jx, T[3]);
                    T[4] = fmaf(mr3, jy, T[4]);
                    T[5] = fmaf(mr3, jz, T[5]);
                    T[6] = fmaf(mr3, fmaf(a6, jx, fmaf(b3, dx, dax)), T[6]);
                    T[7] = fmaf(mr3, fmaf(a6, jy, fmaf(b3, dy, day)), T[7]);
                    T[8] = fmaf(mr3, fmaf(a6, jz, fmaf(b3, dz, daz)), T[8]);
                    continue;
                }
                const double dxd = s_x[t] - xi, dyd = s_y[t] - yi, dzd = s_z[t] - zi;
                const double r2 = fma(dxd, dxd, fma(dyd, dyd, fma(dzd, dzd, eps2)));
                double rinv;
                if constexpr (MIXED)
                    rinv = rinv_mixed(r2);
                else
                    rinv = rinv_f64(r2);
                if constexpr (EPS0)
                    rinv = r2 > 0.0 ? rinv : 0.0;
                const double mrinv = s_m[t] * rinv;
                if constexpr (PHI)
                    phi -= mrinv;
                const double rinv2 = rinv * rinv;
                const double mr3 = mrinv * rinv2;
                if constexpr (MIXED) {
                    // acceleration in FP64; jerk and snap in FP32:
                    // J = m r^-3 (v - 3 alpha r), S = m r^-3 (a - 6 alpha jv - 3 beta r)
                    D[0] = fma(mr3, dxd, D[0]);
                    D[1] = fma(mr3, dyd, D[1]);
                    D[2] = fma(mr3, dzd, D[2]);
                    const float dx = (float)dxd, dy = (float)dyd, dz = (float)dzd;
                    const float fr2 = (float)rinv2, fm3 = (float)mr3;
                    const float dvx = s_vx[t] - vxi, dvy = s_vy[t] - vyi, dvz = s_vz[t] - vzi;
                    const float dax = s_ax[t] - axi, day = s_ay[t] - ayi, daz = s_az[t] - azi;
                    const float rv = fmaf(dx, dvx, fmaf(dy, dvy, dz * dvz));
                    const float qq = fmaf(dvx, dvx, fmaf(dvy, dvy, fmaf(dvz, dvz,
                                     fmaf(dx, dax, fmaf(dy, day, dz * daz)))));
                    const float alpha = rv * fr2;
                    const float beta = fmaf(alpha, alpha, qq * fr2);
                    const float a3 = -3.0f * alpha;
                    const float a6 = a3 + a3;
                    const float b3 = -3.0f * beta;
                    const float jx = fmaf(a3, dx, dvx), jy = fmaf(a3, dy, dvy), jz = fmaf(a3, dz, dvz);
                    const float sx = fmaf(a6, jx, fmaf(b3, dx, dax));
                    const float sy = fmaf(a6, jy, fmaf(b3, dy, day));
                    const float sz = fmaf(a6, jz, fmaf(b3, dz, daz));
                    T[0] = fmaf(fm3, jx, T[0]);
                    T[1] = fmaf(fm3, jy, T[1]);
                    T[2] = fmaf(fm3, jz, T[2]);
                    T[3] = fmaf(fm3, sx, T[3]);
                    T[4] = fmaf(fm3, sy, T[4]);
                    T[5] = fmaf(fm3, sz, T[5]);
                } else {
                    const double dvx = s_vx[t] - vxi, dvy = s_vy[t] - vyi, dvz = s_vz[t] - vzi;
                    const double dax = s_ax[t] - axi, day = s_ay[t] - ayi, daz = s_az[t] - azi;
                    const double alpha = fma(dxd, dvx, fma(dyd, dvy, dzd * dvz)) * rinv2;
                    const double qq = fma(dvx, dvx, fma(dvy, dvy, fma(dvz, dvz,
                                      fma(dxd, dax, fma(dyd, day, dzd * daz)))));
                    const double beta = fma(alpha, alpha, qq * rinv2);
                    if constexpr (INIT) {
                        // start-up evaluation with the crackle, term by term
                        const double djx = s_jx[t] - jxi, djy = s_jy[t] - jyi, djz = s_jz[t] - jzi;
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
                        D[0] += Ax; D[1] += Ay; D[2] += Az;
                        D[3] += Jx; D[4] += Jy; D[5] += Jz;
                        D[6] += Sx; D[7] += Sy; D[8] += Sz;
                        D[ND - 3] += mr3 * djx - 9.0 * alpha * Sx - 9.0 * beta * Jx - 3.0 * gamma * Ax;
                        D[ND - 2] += mr3 * djy - 9.0 * alpha * Sy - 9.0 * beta * Jy - 3.0 * gamma * Ay;
                        D[ND - 1] += mr3 * djz - 9.0 * alpha * Sz - 9.0 * beta * Jz - 3.0 * gamma * Az;
                    } else {
                        const double a3 = -3.0 * alpha, a6 = a3 + a3, b3 = -3.0 * beta;
                        const double jx = fma(a3, dxd, dvx), jy = fma(a3, dyd, dvy), jz = fma(a3, dzd, dvz);
                        D[0] = fma(mr3, dxd, D[0]);
                        D[1] = fma(mr3, dyd, D[1]);
                        D[2] = fma(mr3, dzd, D[2]);
                        D[3] = fma(mr3, jx, D[3]);
                        D[4] = fma(mr3, jy, D[4]);
                        D[5] = fma(mr3, jz, D[5]);
                        D[6] = fma(mr3, fma(a6, jx, fma(b3, dxd, dax)), D[6]);
                        D[7] = fma(mr3, fma(a6, jy, fma(b3, dyd, day)), D[7]);
                        D[8] = fma(mr3, fma(a6, jz, fma(b3, dzd, daz)), D[8]);
                    }
                }
            }
            if constexpr (MIXED || P32) {
#pragma unroll
                for (int q = 0; q < NF; ++q)
                    ds_add(H[q], L[q], T[q]);
            }
        }
    }

    // ---- combine the LPI lanes of each active particle (xor butterfly)
    double R[NV + 1];
    if constexpr (P32) {
#pragma unroll
        for (int q = 0; q < NF; ++q)
            R[q] = (double)H[q] + (double)L[q];
    } else if constexpr (MIXED) {
#pragma unroll
        for (int q = 0; q < 3; ++q)
            R[q] = D[q];
#pragma unroll
        for (int q = 0; q < NF; ++q)
            R[3 + q] = (double)H[q] + (double)L[q];
    } else {
#pragma unroll
        for (int q = 0; q < NV; ++q)
            R[q] = D[q];
    }
    R[NV] = phi;
#pragma unroll
    for (int msk = 1; msk < LPI; msk <<= 1) {
#pragma unroll
        for (int q = 0; q < NV + 1; ++q)
            R[q] += __shfl_xor(R[q], msk, 64);
    }

    if (!valid || js != 0)
        return;
    // the j == i pair adds exactly zero to a, da, d2a but -m_i / eps to the
    // potential: remove that term, computed with the same operations
    if constexpr (!EPS0 && PHI) {
        if (i >= j0 && i < j1) {
            if constexpr (P32) {
                const float e2f = (float)eps2;
                const float ri = __builtin_amdgcn_rsqf(fmaf(0.0f, 0.0f, fmaf(0.0f, 0.0f, fmaf(0.0f, 0.0f, e2f))));
                R[NV] += (double)((float)J.m[i] * ri);
            } else {
                const double r2 = fma(0.0, 0.0, fma(0.0, 0.0, fma(0.0, 0.0, eps2)));
                const double ri = MIXED ? rinv_mixed(r2) : rinv_f64(r2);
                R[NV] += J.m[i] * ri;
            }
        }
    }
    if constexpr (INIT) {
#pragma unroll
        for (int q = 0; q < NV / 3; ++q)
            if (out.vec[q])
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    out.vec[q][k * out.sk + d * out.sd] = R[3 * q + d];
        return;
    }
    if (part) {
        double *pb = part + (int64_t)b * 10 * n_act_total + k;
#pragma unroll
        for (int q = 0; q < 10; ++q)
            pb[(int64_t)q * n_act_total] = R[q];
    } else {
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int d = 0; d < 3; ++d)
                out.vec[q][k * out.sk + d * out.sd] = R[3 * q + d];
        if (out.pot)
            out.pot[k] = R[NV];
    }
}

}  // namespace

}  // namespace nb
