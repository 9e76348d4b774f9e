/*
 * nbody_oracle.c -- plain FP64 CPU oracle for the block-time-step,
 * sixth-order Hermite direct-summation N-body method of
 * Capuzzo-Dolcetta, Spera & Punzo, "A fully parallel, high precision,
 * N-body code running on hybrid computing platforms" (arXiv:1207.2367).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or helper with the HIP library.
 *
 * Conventions
 *   - every vector array is row-major [n][3] (x, y, z of a particle adjacent);
 *   - G = 1 (paper, Sect. 5: b = M = G = 1 units; the inputs here use
 *     Henon units, which also have G = M = 1);
 *   - arithmetic is IEEE binary64, compiled without FMA contraction and
 *     without fast-math; every force sum runs over the source index j in
 *     ascending order; OpenMP splits the work over active particles only,
 *     so results do not depend on the thread count.
 *
 * Readings of the paper that this file fixes (the paper is silent or
 * ambiguous on them) are marked "READING" below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENONFINITE (-3)
#define ORC_EDTMIN (-4)

/* ------------------------------------------------------------------ */
/* O1. Evaluation step (paper Sect. 3, item 2, the three sums for     */
/* a_{i,1}, da_{i,1}, d2a_{i,1}) with Plummer softening (Sect. 2,     */
/* Eq. softpot).                                                      */
/*                                                                    */
/* For each listed particle i and every source j in [j0, j1), j != i: */
/*   r = r_j - r_i, v = v_j - v_i, a = a_j - a_i   (predicted values) */
/*   alpha r^2 = r.v ; beta r^2 = v.v + r.a + alpha^2 r^2             */
/*   A = m_j r / r^3                                                  */
/*   J = m_j v / r^3 - 3 alpha A                                      */
/*   S = m_j a / r^3 - 6 alpha J - 3 beta A                           */
/*   phi_i -= m_j / r                                                 */
/* READING: the softened distance r^2 + eps^2 replaces r^2 in every   */
/* one of these terms (the softened pair acceleration and its two     */
/* time derivatives are then exact derivatives of each other).        */
/* READING: alpha in the snap term is alpha_ij (missing subscript).   */
/* READING: the j == i term is excluded by index, so a distinct       */
/* particle at the same place still contributes to phi when eps > 0.  */
/* ------------------------------------------------------------------ */
void orc_force(int64_t n, const double *m, const double *x, const double *v,
               const double *a, double eps, int64_t j0, int64_t j1,
               int64_t n_act, const int64_t *idx, double *acc, double *jrk,
               double *snp, double *pot)
{
    const double eps2 = eps * eps;
    (void)n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n_act; ++k) {
        const int64_t i = idx[k];
        double ai[3] = {0, 0, 0}, ji[3] = {0, 0, 0}, si[3] = {0, 0, 0};
        double phi = 0.0;
        for (int64_t j = j0; j < j1; ++j) {
            if (j == i)
                continue;
            double r[3], w[3], q[3];
            for (int d = 0; d < 3; ++d) {
                r[d] = x[3 * j + d] - x[3 * i + d];
                w[d] = v[3 * j + d] - v[3 * i + d];
                q[d] = a[3 * j + d] - a[3 * i + d];
            }
            const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps2;
            const double rinv = 1.0 / sqrt(r2);
            const double rinv2 = rinv * rinv;
            const double mr3 = m[j] * rinv * rinv2;
            const double rv = r[0] * w[0] + r[1] * w[1] + r[2] * w[2];
            const double vv = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
            const double ra = r[0] * q[0] + r[1] * q[1] + r[2] * q[2];
            const double alpha = rv * rinv2;
            const double beta = (vv + ra) * rinv2 + alpha * alpha;
            for (int d = 0; d < 3; ++d) {
                const double A = mr3 * r[d];
                const double J = mr3 * w[d] - 3.0 * alpha * A;
                const double S = mr3 * q[d] - 6.0 * alpha * J - 3.0 * beta * A;
                ai[d] += A;
                ji[d] += J;
                si[d] += S;
            }
            phi -= m[j] * rinv;
        }
        for (int d = 0; d < 3; ++d) {
            acc[3 * k + d] = ai[d];
            jrk[3 * k + d] = ji[d];
            snp[3 * k + d] = si[d];
        }
        pot[k] = phi;
    }
}

/* ------------------------------------------------------------------ */
/* O1'. The same sums and, in addition, the crackle (third derivative  */
/* of the acceleration), needed once at the start (O7).  It is the    */
/* time derivative of the snap term along the trajectories, with the  */
/* sources' jerks j_j entering through q = j_j - j_i:                 */
/*   gamma r^2 = 3 v.a + r.q + alpha (3 beta - 4 alpha^2) r^2         */
/*   C = m_j q / r^3 - 9 alpha S - 9 beta J - 3 gamma A               */
/* (softened distance throughout, as in O1).                          */
/* ------------------------------------------------------------------ */
void orc_force4(int64_t n, const double *m, const double *x, const double *v,
                const double *a, const double *jk, double eps, int64_t j0,
                int64_t j1, int64_t n_act, const int64_t *idx, double *acc,
                double *jrk, double *snp, double *crk)
{
    const double eps2 = eps * eps;
    (void)n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n_act; ++k) {
        const int64_t i = idx[k];
        double ai[3] = {0, 0, 0}, ji[3] = {0, 0, 0}, si[3] = {0, 0, 0};
        double ci[3] = {0, 0, 0};
        for (int64_t j = j0; j < j1; ++j) {
            if (j == i)
                continue;
            double r[3], w[3], q[3], u[3];
            for (int d = 0; d < 3; ++d) {
                r[d] = x[3 * j + d] - x[3 * i + d];
                w[d] = v[3 * j + d] - v[3 * i + d];
                q[d] = a[3 * j + d] - a[3 * i + d];
                u[d] = jk[3 * j + d] - jk[3 * i + d];
            }
            const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps2;
            const double rinv = 1.0 / sqrt(r2);
            const double rinv2 = rinv * rinv;
            const double mr3 = m[j] * rinv * rinv2;
            const double rv = r[0] * w[0] + r[1] * w[1] + r[2] * w[2];
            const double vv = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
            const double ra = r[0] * q[0] + r[1] * q[1] + r[2] * q[2];
            const double va = w[0] * q[0] + w[1] * q[1] + w[2] * q[2];
            const double rj = r[0] * u[0] + r[1] * u[1] + r[2] * u[2];
            const double alpha = rv * rinv2;
            const double beta = (vv + ra) * rinv2 + alpha * alpha;
            const double gamma =
                (3.0 * va + rj) * rinv2 + alpha * (3.0 * beta - 4.0 * alpha * alpha);
            for (int d = 0; d < 3; ++d) {
                const double A = mr3 * r[d];
                const double J = mr3 * w[d] - 3.0 * alpha * A;
                const double S = mr3 * q[d] - 6.0 * alpha * J - 3.0 * beta * A;
                const double Cc = mr3 * u[d] - 9.0 * alpha * S - 9.0 * beta * J -
                                  3.0 * gamma * A;
                ai[d] += A;
                ji[d] += J;
                si[d] += S;
                ci[d] += Cc;
            }
        }
        for (int d = 0; d < 3; ++d) {
            acc[3 * k + d] = ai[d];
            jrk[3 * k + d] = ji[d];
            snp[3 * k + d] = si[d];
            crk[3 * k + d] = ci[d];
        }
    }
}

/* ------------------------------------------------------------------ */
/* O2. Prediction step (paper Sect. 3, item 1): Taylor series of      */
/* position to the crackle term, velocity to the crackle term and     */
/* acceleration to the crackle term.                                  */
/* READING: the step length in the series is, per particle, the time  */
/* elapsed since its last correction, h = T - t_i.                    */
/* ------------------------------------------------------------------ */
void orc_predict(int64_t n, const double *x, const double *v, const double *a,
                 const double *jk, const double *sn, const double *cr,
                 const double *t, double T, double *xp, double *vp, double *ap)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double h = T - t[i];
        const double h2 = h * h, h3 = h2 * h, h4 = h3 * h, h5 = h4 * h;
        for (int d = 0; d < 3; ++d) {
            const int64_t e = 3 * i + d;
            xp[e] = x[e] + v[e] * h + a[e] * h2 / 2.0 + jk[e] * h3 / 6.0 +
                    sn[e] * h4 / 24.0 + cr[e] * h5 / 120.0;
            vp[e] = v[e] + a[e] * h + jk[e] * h2 / 2.0 + sn[e] * h3 / 6.0 +
                    cr[e] * h4 / 24.0;
            ap[e] = a[e] + jk[e] * h + sn[e] * h2 / 2.0 + cr[e] * h3 / 6.0;
        }
    }
}

/* ------------------------------------------------------------------ */
/* O5. Higher derivatives at the end of a step.  The paper uses the   */
/* crackle in the predictor and derivatives up to the fifth in the    */
/* time-step criterion but does not say how they are obtained.        */
/* READING: they are the derivatives of the unique quintic that       */
/* matches a, da, d2a at both ends of the step (the same polynomial   */
/* that makes the corrector exact).  Writing it as a Taylor series    */
/* about the start of the step,                                       */
/*   a(tau) = a0 + j0 tau + s0 tau^2/2 + c tau^3/6 + p tau^4/24       */
/*            + x tau^5/120,                                          */
/* the three end conditions fix C = c h^3, P = p h^4, X = x h^5 from  */
/*   D0 = a1 - a0 - h j0 - h^2 s0 / 2,  D1 = j1 - j0 - h s0,          */
/*   D2 = s1 - s0:                                                    */
/*   C =   60 D0 -  24 h D1 +  3 h^2 D2                               */
/*   P = -360 D0 + 168 h D1 - 24 h^2 D2                               */
/*   X =  720 D0 - 360 h D1 + 60 h^2 D2                               */
/* and the derivatives at the end are c + p h + x h^2/2, p + x h, x.  */
/* ------------------------------------------------------------------ */
void orc_interpolate(double h, const double *a0, const double *j0,
                     const double *s0, const double *a1, const double *j1,
                     const double *s1, double *crk1, double *pop1, double *a51)
{
    for (int d = 0; d < 3; ++d) {
        const double D0 = a1[d] - a0[d] - h * j0[d] - h * h * s0[d] / 2.0;
        const double D1 = j1[d] - j0[d] - h * s0[d];
        const double D2 = s1[d] - s0[d];
        const double C = 60.0 * D0 - 24.0 * h * D1 + 3.0 * h * h * D2;
        const double P = -360.0 * D0 + 168.0 * h * D1 - 24.0 * h * h * D2;
        const double X = 720.0 * D0 - 360.0 * h * D1 + 60.0 * h * h * D2;
        const double c = C / (h * h * h);
        const double p = P / (h * h * h * h);
        const double xx = X / (h * h * h * h * h);
        crk1[d] = c + p * h + xx * h * h / 2.0;
        pop1[d] = p + xx * h;
        a51[d] = xx;
    }
}

static double norm3(const double *u)
{
    return sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
}

/* ------------------------------------------------------------------ */
/* O6. Generalized Aarseth criterion (paper Sect. 3, Eqs. indtstp and */
/* As) with p = 6:                                                    */
/*   A(1) = sqrt(|a||d2a| + |da|^2),                                  */
/*   A(4) = sqrt(|a(3)||a(5)| + |a(4)|^2),                            */
/*   dt = eta (A(1)/A(4))^(1/3).                                      */
/* READING (degenerate cases): A(4) = 0 gives +inf (clamped to the    */
/* maximum step by the block rules); A(1) = 0 with A(4) > 0 gives 0.  */
/* ------------------------------------------------------------------ */
double orc_dt_criterion(const double *a, const double *jk, const double *sn,
                        const double *cr, const double *pp, const double *a5,
                        double eta)
{
    const double A1 = sqrt(norm3(a) * norm3(sn) + norm3(jk) * norm3(jk));
    const double A4 = sqrt(norm3(cr) * norm3(a5) + norm3(pp) * norm3(pp));
    if (A4 == 0.0)
        return INFINITY;
    return eta * cbrt(A1 / A4);
}

/* ------------------------------------------------------------------ */
/* O8. Block (power-of-two) time-step rules.  The paper fixes only    */
/* that steps are quantized to powers of two between a minimum and a  */
/* maximum (Sect. 3, after Eq. As).  READING of the rest:             */
/*  (i)  round the criterion down to a power of two, clamp to         */
/*       [dt_min, dt_max];                                            */
/*  (ii) a larger step is accepted only as a doubling, and only when  */
/*       the new time is a multiple of twice the old step;            */
/*  (iii) a smaller step is always accepted;                          */
/*  (iv) while the particle is short of t_target, halve the step      */
/*       while it would pass t_target (a particle that has arrived     */
/*       keeps its step; a later run re-caps it, see orc_recap);       */
/*  (v)  a criterion below dt_min, or a cap below dt_min, is an error */
/*       (the step would not resolve the orbit).                      */
/* dt_old <= 0 means "no previous step" (initialization).             */
/* All times are dyadic rationals >= dt_min, so every comparison and  */
/* fmod below is exact in binary64.                                   */
/* ------------------------------------------------------------------ */
int orc_block_dt(double dt_crit, double dt_old, double t_new, double t_target,
                 double dt_min, double dt_max, double *dt_out)
{
    if (isnan(dt_crit))
        return ORC_ENONFINITE;
    if (dt_crit < dt_min)
        return ORC_EDTMIN;
    double dt = dt_max;
    if (dt_crit < dt_max) {
        /* largest power of two <= dt_crit */
        int e;
        const double f = frexp(dt_crit, &e); /* dt_crit = f 2^e, f in [0.5,1) */
        (void)f;
        dt = ldexp(1.0, e - 1);
        if (dt < dt_min)
            dt = dt_min;
    }
    if (dt_old > 0.0 && dt > dt_old) {
        if (fmod(t_new, 2.0 * dt_old) == 0.0 && 2.0 * dt_old <= dt_max)
            dt = 2.0 * dt_old;
        else
            dt = dt_old;
    }
    if (t_new < t_target)
        while (t_new + dt > t_target)
            dt *= 0.5;
    if (dt < dt_min)
        return ORC_EDTMIN;
    *dt_out = dt;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* O9. Active-set selection (paper Sect. 5.4, Table 1, section 1):    */
/* the next block time is the smallest t_i + dt_i; the active         */
/* particles are those due exactly then, listed in ascending index.   */
/* ------------------------------------------------------------------ */
void orc_schedule(int64_t n, const double *t, const double *dt, int64_t *idx,
                  int64_t *n_act, double *t_next)
{
    double tn = INFINITY;
    for (int64_t i = 0; i < n; ++i)
        if (t[i] + dt[i] < tn)
            tn = t[i] + dt[i];
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i)
        if (t[i] + dt[i] == tn)
            idx[k++] = i;
    *n_act = k;
    *t_next = tn;
}

/* ------------------------------------------------------------------ */
/* Integrator state.                                                  */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    double *m;                          /* [n]     */
    double *x, *v, *a, *jk, *sn, *cr;   /* [n][3]  */
    double *t, *dt;                     /* [n]     */
    double eps, eta, eta_init, dt_min, dt_max;
} orc_state;

/* ------------------------------------------------------------------ */
/* O4 + O5 + O6 + O8 for the listed particles.  Corrector of paper    */
/* Sect. 3, item 3 (velocity first, then position with the corrected  */
/* velocity), with h = t_new - t_i (the particle's own step).         */
/* ------------------------------------------------------------------ */
int orc_correct(orc_state *st, int64_t n_act, const int64_t *idx, double t_new,
                double t_target, const double *acc1, const double *jrk1,
                const double *snp1)
{
    int err = ORC_OK;
#pragma omp parallel for schedule(static) reduction(min : err)
    for (int64_t k = 0; k < n_act; ++k) {
        const int64_t i = idx[k];
        const double h = t_new - st->t[i];
        const double *a0 = st->a + 3 * i, *j0 = st->jk + 3 * i,
                     *s0 = st->sn + 3 * i;
        const double *a1 = acc1 + 3 * k, *j1 = jrk1 + 3 * k, *s1 = snp1 + 3 * k;
        double v1[3], r1[3];
        for (int d = 0; d < 3; ++d) {
            const double v0 = st->v[3 * i + d], r0 = st->x[3 * i + d];
            v1[d] = v0 + h / 2.0 * (a1[d] + a0[d]) -
                    h * h / 10.0 * (j1[d] - j0[d]) +
                    h * h * h / 120.0 * (s1[d] + s0[d]);
            r1[d] = r0 + h / 2.0 * (v1[d] + v0) -
                    h * h / 10.0 * (a1[d] - a0[d]) +
                    h * h * h / 120.0 * (j1[d] + j0[d]);
        }
        double crk1[3], pop1[3], a51[3];
        orc_interpolate(h, a0, j0, s0, a1, j1, s1, crk1, pop1, a51);
        const double dtc =
            orc_dt_criterion(a1, j1, s1, crk1, pop1, a51, st->eta);
        double dtn = 0.0;
        int e = orc_block_dt(dtc, st->dt[i], t_new, t_target, st->dt_min,
                             st->dt_max, &dtn);
        for (int d = 0; d < 3; ++d) {
            st->x[3 * i + d] = r1[d];
            st->v[3 * i + d] = v1[d];
            st->a[3 * i + d] = a1[d];
            st->jk[3 * i + d] = j1[d];
            st->sn[3 * i + d] = s1[d];
            st->cr[3 * i + d] = crk1[d];
            if (!isfinite(r1[d]) || !isfinite(v1[d]))
                e = ORC_ENONFINITE;
        }
        st->t[i] = t_new;
        if (e == ORC_OK)
            st->dt[i] = dtn;
        if (e < err)
            err = e;
    }
    return err;
}

/* ------------------------------------------------------------------ */
/* O7. Initialization (the paper does not describe it).  READING:     */
/* pass 1 evaluates a and da with zero source accelerations (they do  */
/* not enter a or da); pass 2 evaluates d2a and the crackle with the  */
/* pass-1 accelerations and jerks as the sources' values (O1').  With */
/* every derivative up to the crackle known, the first step is the    */
/* paper's generalized criterion (Eqs. indtstp, As) at the order the   */
/* known derivatives allow, p = 4: dt = eta_init A(1) / A(2), with     */
/* A(2) = sqrt(|da||a(3)| + |d2a|^2), then the block rules; t_i = 0.   */
/* Sources are the particles of the particle's own cluster, given by  */
/* offsets[0..n_clusters] (pairs across clusters do not interact).    */
/* ------------------------------------------------------------------ */
static int64_t cluster_of(int64_t i, int64_t nc, const int64_t *off)
{
    int64_t lo = 0, hi = nc; /* off[lo] <= i < off[hi] */
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (off[mid] <= i)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

static void force_clusters(orc_state *st, const double *x, const double *v,
                           const double *a, const double *jk, int64_t n_act,
                           const int64_t *idx, int64_t nc, const int64_t *off,
                           double *acc, double *jrk, double *snp, double *pot,
                           double *crk)
{
    /* active lists are ascending, so each cluster's actives are contiguous */
    int64_t k = 0;
    while (k < n_act) {
        const int64_t c = cluster_of(idx[k], nc, off);
        int64_t k1 = k;
        while (k1 < n_act && idx[k1] < off[c + 1])
            ++k1;
        if (crk)
            orc_force4(st->n, st->m, x, v, a, jk, st->eps, off[c], off[c + 1],
                       k1 - k, idx + k, acc + 3 * k, jrk + 3 * k, snp + 3 * k,
                       crk + 3 * k);
        else
            orc_force(st->n, st->m, x, v, a, st->eps, off[c], off[c + 1], k1 - k,
                      idx + k, acc + 3 * k, jrk + 3 * k, snp + 3 * k, pot + k);
        k = k1;
    }
}

int orc_init(orc_state *st, int64_t nc, const int64_t *off, double t_target)
{
    const int64_t n = st->n;
    int64_t *all = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    double *zero = (double *)calloc((size_t)(3 * n), sizeof(double));
    double *pot = (double *)malloc(sizeof(double) * (size_t)n);
    if (!all || !zero || !pot) {
        free(all); free(zero); free(pot);
        return ORC_EINVAL;
    }
    for (int64_t i = 0; i < n; ++i)
        all[i] = i;
    force_clusters(st, st->x, st->v, zero, zero, n, all, nc, off, st->a, st->jk,
                   st->sn, pot, NULL);
    double *a1 = (double *)malloc(sizeof(double) * (size_t)(6 * n));
    if (!a1) {
        free(all); free(zero); free(pot);
        return ORC_EINVAL;
    }
    memcpy(a1, st->a, sizeof(double) * (size_t)(3 * n));
    memcpy(a1 + 3 * n, st->jk, sizeof(double) * (size_t)(3 * n));
    force_clusters(st, st->x, st->v, a1, a1 + 3 * n, n, all, nc, off, st->a,
                   st->jk, st->sn, pot, st->cr);
    free(a1);
    int err = ORC_OK;
    for (int64_t i = 0; i < n; ++i) {
        st->t[i] = 0.0;
        const double A1 = sqrt(norm3(st->a + 3 * i) * norm3(st->sn + 3 * i) +
                               norm3(st->jk + 3 * i) * norm3(st->jk + 3 * i));
        const double A2 = sqrt(norm3(st->jk + 3 * i) * norm3(st->cr + 3 * i) +
                               norm3(st->sn + 3 * i) * norm3(st->sn + 3 * i));
        const double dtc = (A2 > 0.0) ? st->eta_init * A1 / A2 : INFINITY;
        double dtn = 0.0;
        const int e = orc_block_dt(dtc, 0.0, 0.0, t_target, st->dt_min,
                                   st->dt_max, &dtn);
        if (e != ORC_OK && e < err)
            err = e;
        st->dt[i] = dtn;
    }
    free(all); free(zero); free(pot);
    return err;
}

/* ------------------------------------------------------------------ */
/* One block step of the Hermite scheme (paper Sect. 3 items 1-3 in   */
/* the order of Table 1): select the active block (per cluster, each  */
/* cluster at its own block time), predict every source to that time, */
/* evaluate the active particles, correct them and give them new      */
/* steps.  Clusters whose particles have all reached t_target are     */
/* left alone.  Returns the number of active particles in *n_act.     */
/* ------------------------------------------------------------------ */
int orc_block_step(orc_state *st, int64_t nc, const int64_t *off,
                   double t_target, int64_t *n_act_out, double *t_block_out)
{
    const int64_t n = st->n;
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    double *xp = (double *)malloc(sizeof(double) * (size_t)(9 * n));
    double *out = (double *)malloc(sizeof(double) * (size_t)(10 * n));
    double *tb = (double *)malloc(sizeof(double) * (size_t)nc);
    if (!idx || !xp || !out || !tb) {
        free(idx); free(xp); free(out); free(tb);
        return ORC_EINVAL;
    }
    double *vp = xp + 3 * n, *ap = xp + 6 * n;
    int64_t na = 0;
    double tmin = INFINITY;
    for (int64_t c = 0; c < nc; ++c) {
        int64_t k = 0;
        double tn = 0.0;
        const int64_t o = off[c], nn = off[c + 1] - off[c];
        orc_schedule(nn, st->t + o, st->dt + o, idx + na, &k, &tn);
        tb[c] = tn;
        if (!(tn <= t_target)) /* cluster done (or empty) */
            continue;
        for (int64_t q = 0; q < k; ++q)
            idx[na + q] += o;
        /* predict the cluster's sources to its block time */
        orc_predict(nn, st->x + 3 * o, st->v + 3 * o, st->a + 3 * o,
                    st->jk + 3 * o, st->sn + 3 * o, st->cr + 3 * o, st->t + o,
                    tn, xp + 3 * o, vp + 3 * o, ap + 3 * o);
        if (tn < tmin)
            tmin = tn;
        na += k;
    }
    int err = ORC_OK;
    if (na > 0) {
        double *acc = out, *jrk = out + 3 * na, *snp = out + 6 * na,
               *pot = out + 9 * na;
        force_clusters(st, xp, vp, ap, NULL, na, idx, nc, off, acc, jrk, snp, pot,
                       NULL);
        /* correct each cluster's block at its own block time */
        int64_t k = 0;
        while (k < na) {
            const int64_t c = cluster_of(idx[k], nc, off);
            int64_t k1 = k;
            while (k1 < na && idx[k1] < off[c + 1])
                ++k1;
            const int e = orc_correct(st, k1 - k, idx + k, tb[c], t_target,
                                      acc + 3 * k, jrk + 3 * k, snp + 3 * k);
            if (e < err)
                err = e;
            k = k1;
        }
    }
    *n_act_out = na;
    *t_block_out = tmin;
    free(idx); free(xp); free(out); free(tb);
    return err;
}

/* Rule (iv) at the start of a run: a particle short of the new target */
/* whose step would pass it halves the step until it does not (t_i is  */
/* a multiple of dt_i and t_target of dt_min, so this ends >= dt_min). */
void orc_recap(orc_state *st, double t_target)
{
    for (int64_t i = 0; i < st->n; ++i)
        if (st->t[i] < t_target)
            while (st->t[i] + st->dt[i] > t_target)
                st->dt[i] *= 0.5;
}

/* Advance every cluster to t_target.  *steps and *pairs count block   */
/* steps and interactions (N_cluster * N_act summed over steps).       */
int orc_run(orc_state *st, int64_t nc, const int64_t *off, double t_target,
            int64_t *steps, double *pairs, int64_t *hist /* [64] or NULL */)
{
    int64_t s = 0;
    double p = 0.0;
    orc_recap(st, t_target);
    for (;;) {
        int done = 1;
        for (int64_t i = 0; i < st->n; ++i)
            if (st->t[i] < t_target) {
                done = 0;
                break;
            }
        if (done)
            break;
        /* count interactions before the step: N_c of each active cluster */
        int64_t na = 0;
        double tb = 0.0;
        int64_t *cnt = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
        for (int64_t c = 0; c < nc; ++c) {
            double tn = INFINITY;
            for (int64_t i = off[c]; i < off[c + 1]; ++i)
                if (st->t[i] + st->dt[i] < tn)
                    tn = st->t[i] + st->dt[i];
            if (tn <= t_target)
                for (int64_t i = off[c]; i < off[c + 1]; ++i)
                    if (st->t[i] + st->dt[i] == tn)
                        ++cnt[c];
        }
        for (int64_t c = 0; c < nc; ++c) {
            p += (double)cnt[c] * (double)(off[c + 1] - off[c]);
            if (hist && cnt[c] > 0) {
                int b = 0;
                while ((INT64_C(1) << (b + 1)) <= cnt[c])
                    ++b;
                hist[b] += 1;
            }
        }
        free(cnt);
        const int e = orc_block_step(st, nc, off, t_target, &na, &tb);
        ++s;
        if (e != ORC_OK) {
            *steps = s;
            *pairs = p;
            return e;
        }
        if (na == 0)
            break;
    }
    *steps = s;
    *pairs = p;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* O10. Energy and angular momentum (paper Sect. 5.1): kinetic energy */
/* sum m v^2 / 2, softened potential energy -sum_{i<j} m_i m_j /      */
/* sqrt(r^2 + eps^2) (READING: the softened potential is the one the  */
/* integrated dynamics conserves), and L = sum m r x v.  Pairs across */
/* clusters are not counted.                                          */
/* ------------------------------------------------------------------ */
void orc_energy(int64_t n, const double *m, const double *x, const double *v,
                double eps, int64_t nc, const int64_t *off, double *ekin,
                double *epot, double *L)
{
    double *w = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    const double eps2 = eps * eps;
    for (int64_t c = 0; c < nc; ++c) {
        const int64_t j1 = off[c + 1];
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = off[c]; i < j1; ++i) {
            double s = 0.0;
            for (int64_t j = i + 1; j < j1; ++j) {
                const double dx = x[3 * j] - x[3 * i];
                const double dy = x[3 * j + 1] - x[3 * i + 1];
                const double dz = x[3 * j + 2] - x[3 * i + 2];
                s += m[i] * m[j] / sqrt(dx * dx + dy * dy + dz * dz + eps2);
            }
            w[i] = s;
        }
    }
    double k = 0.0, u = 0.0, lx = 0.0, ly = 0.0, lz = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double *r = x + 3 * i, *u3 = v + 3 * i;
        k += 0.5 * m[i] * (u3[0] * u3[0] + u3[1] * u3[1] + u3[2] * u3[2]);
        u -= w[i];
        lx += m[i] * (r[1] * u3[2] - r[2] * u3[1]);
        ly += m[i] * (r[2] * u3[0] - r[0] * u3[2]);
        lz += m[i] * (r[0] * u3[1] - r[1] * u3[0]);
    }
    *ekin = k;
    *epot = u;
    L[0] = lx;
    L[1] = ly;
    L[2] = lz;
    free(w);
}
