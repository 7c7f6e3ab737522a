/*
 * Plain FP64 CPU oracle for softened direct-sum gravity.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is used by the test-suite, by the smoke
 * check and by the CPU-baseline leg of the benchmark; nothing in the product
 * library links or calls it, and it includes nothing from the product.  It is
 * deliberately slow and obvious: one loop over i, one loop over j, IEEE sqrt and
 * division in double precision, no blocking and no reordering.  OpenMP only
 * splits the outer i loop across threads, which does not change any sum.
 *
 * Arrays are row-major "array of structures": positions are n x 3 doubles
 * (x0 y0 z0 x1 y1 z1 ...).  G = 1.
 *
 * Definitions (Hamada & Iitaka, Sec. 1.1, eq. (1); the potential is the
 * quantity accumulated by the force-jerk-potential pipeline of Appendix A):
 *   d_ij  = x_j - x_i
 *   s_ij  = sqrt(|d_ij|^2 + eps^2)
 *   a_i   =  sum_{j != i} m_j d_ij / s_ij^3
 *   phi_i = -sum_{j != i} m_j / s_ij
 * The self pair j == i is excluded (eq. (1) is silent; with eps > 0 the self
 * term of a is zero and the self term of phi is -m_i/eps).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------- */
/* Forces and potentials of a set of i-particles from a set of j-particles.   */
/* eq. (1): a_i = sum_j m_j r_ij / (r_ij^2 + eps^2)^{3/2}.                     */
/* self[i] is the j index to skip for i (the same particle), or -1; self may  */
/* be NULL when no j is to be skipped.  pot may be NULL.                      */
/* ------------------------------------------------------------------------- */
OR_EXPORT void oracle_force(int64_t nj, const double *xj, const double *mj,
                            int64_t ni, const double *xi, const int64_t *self,
                            double eps, double *acc, double *pot)
{
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < ni; ++i) {
        const int64_t skip = self ? self[i] : -1;
        double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
        for (int64_t j = 0; j < nj; ++j) {
            if (j == skip)
                continue;
            const double dx = xj[3 * j + 0] - xi[3 * i + 0];
            const double dy = xj[3 * j + 1] - xi[3 * i + 1];
            const double dz = xj[3 * j + 2] - xi[3 * i + 2];
            const double s2 = dx * dx + dy * dy + dz * dz + eps2;
            const double s = sqrt(s2);
            const double s3 = s2 * s;
            ax += mj[j] * dx / s3;
            ay += mj[j] * dy / s3;
            az += mj[j] * dz / s3;
            ph -= mj[j] / s;
        }
        acc[3 * i + 0] = ax;
        acc[3 * i + 1] = ay;
        acc[3 * i + 2] = az;
        if (pot)
            pot[i] = ph;
    }
}

/* Separate i- and j-sets with a softening length per i-particle (the paper's
 * library takes separate i and j arrays, Sec. 3.1, and its driver keeps eps^2 per
 * i-particle, Appendix A).  Every pair is summed; eps_i[i] may be 0. */
OR_EXPORT void oracle_force_epsi(int64_t nj, const double *xj, const double *mj,
                                 int64_t ni, const double *xi, const double *eps_i,
                                 double *acc, double *pot)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < ni; ++i) {
        const double eps2 = eps_i[i] * eps_i[i];
        double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
        for (int64_t j = 0; j < nj; ++j) {
            const double dx = xj[3 * j + 0] - xi[3 * i + 0];
            const double dy = xj[3 * j + 1] - xi[3 * i + 1];
            const double dz = xj[3 * j + 2] - xi[3 * i + 2];
            const double s2 = dx * dx + dy * dy + dz * dz + eps2;
            const double s = sqrt(s2);
            const double s3 = s2 * s;
            ax += mj[j] * dx / s3;
            ay += mj[j] * dy / s3;
            az += mj[j] * dz / s3;
            ph -= mj[j] / s;
        }
        acc[3 * i + 0] = ax;
        acc[3 * i + 1] = ay;
        acc[3 * i + 2] = az;
        if (pot)
            pot[i] = ph;
    }
}

/* Magnitude sums of the terms of eq. (1) and of the potential, for rounding-error   */
/* bounds: absa[3 i + c] = sum_j |m_j d_c| / s^3 and absp[i] = sum_j |m_j| / s, over  */
/* the same pairs as oracle_force (self[i] skipped; self may be NULL).  With         */
/* positive masses and every d_c of one sign, absa is |a_c|; absp is |phi| always.   */
OR_EXPORT void oracle_force_abs(int64_t nj, const double *xj, const double *mj,
                                int64_t ni, const double *xi, const int64_t *self,
                                double eps, double *absa, double *absp)
{
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < ni; ++i) {
        const int64_t skip = self ? self[i] : -1;
        double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
        for (int64_t j = 0; j < nj; ++j) {
            if (j == skip)
                continue;
            const double dx = xj[3 * j + 0] - xi[3 * i + 0];
            const double dy = xj[3 * j + 1] - xi[3 * i + 1];
            const double dz = xj[3 * j + 2] - xi[3 * i + 2];
            const double s2 = dx * dx + dy * dy + dz * dz + eps2;
            const double s = sqrt(s2);
            const double s3 = s2 * s;
            const double mm = fabs(mj[j]);
            ax += mm * fabs(dx) / s3;
            ay += mm * fabs(dy) / s3;
            az += mm * fabs(dz) / s3;
            ph += mm / s;
        }
        absa[3 * i + 0] = ax;
        absa[3 * i + 1] = ay;
        absa[3 * i + 2] = az;
        if (absp)
            absp[i] = ph;
    }
}

/* All-pairs convenience: i-set == j-set, self pair excluded. */
OR_EXPORT void oracle_force_all(int64_t n, const double *x, const double *m,
                                double eps, double *acc, double *pot)
{
    int64_t *self = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i)
        self[i] = i;
    oracle_force(n, x, m, n, x, self, eps, acc, pot);
    free(self);
}

/* Sampled: forces on the listed particles (idx[0..k)) from all n particles. */
OR_EXPORT void oracle_force_sampled(int64_t n, const double *x, const double *m,
                                    double eps, int64_t k, const int64_t *idx,
                                    double *acc, double *pot)
{
    double *xi = (double *)malloc(sizeof(double) * 3 * (size_t)(k > 0 ? k : 1));
    for (int64_t t = 0; t < k; ++t)
        memcpy(xi + 3 * t, x + 3 * idx[t], 3 * sizeof(double));
    oracle_force(n, x, m, k, xi, idx, eps, acc, pot);
    free(xi);
}

/* ------------------------------------------------------------------------- */
/* Force, jerk and potential (the force-jerk-potential pipeline of Appendix A, */
/* the interaction a fourth-order Hermite integrator needs, Sec. 4.1).  With   */
/* d = x_j - x_i, w = v_j - v_i and s^2 = |d|^2 + eps^2, the time derivative   */
/* of the pair acceleration m_j d / s^3 along the motion is                     */
/*   jerk_ij = m_j ( w / s^3 - 3 (d . w) d / s^5 ).                              */
/* self[i] is the j to skip for i, or -1; self may be NULL.  pot may be NULL.   */
/* ------------------------------------------------------------------------- */
OR_EXPORT void oracle_force_jerk(int64_t nj, const double *xj, const double *vj,
                                 const double *mj, int64_t ni, const double *xi,
                                 const double *vi, const int64_t *self, double eps,
                                 double *acc, double *jerk, double *pot)
{
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < ni; ++i) {
        const int64_t skip = self ? self[i] : -1;
        double a[3] = {0.0, 0.0, 0.0}, jk[3] = {0.0, 0.0, 0.0}, ph = 0.0;
        for (int64_t j = 0; j < nj; ++j) {
            if (j == skip)
                continue;
            double d[3], w[3];
            for (int c = 0; c < 3; ++c) {
                d[c] = xj[3 * j + c] - xi[3 * i + c];
                w[c] = vj[3 * j + c] - vi[3 * i + c];
            }
            const double s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
            const double s = sqrt(s2);
            const double s3 = s2 * s;
            const double s5 = s3 * s2;
            const double dw = d[0] * w[0] + d[1] * w[1] + d[2] * w[2];
            for (int c = 0; c < 3; ++c) {
                a[c] += mj[j] * d[c] / s3;
                jk[c] += mj[j] * (w[c] / s3 - 3.0 * dw * d[c] / s5);
            }
            ph -= mj[j] / s;
        }
        for (int c = 0; c < 3; ++c) {
            acc[3 * i + c] = a[c];
            jerk[3 * i + c] = jk[c];
        }
        if (pot)
            pot[i] = ph;
    }
}

/* ------------------------------------------------------------------------- */
/* Vector-Jacobian product of (a, phi) with respect to (x, m).                */
/*                                                                           */
/* Given cotangents ga_i = dL/da_i and gp_i = dL/dphi_i, differentiating the  */
/* definitions above term by term gives, with d = d_kj, s = s_kj and          */
/* K_kj = I/s^3 - 3 d d^T / s^5 (symmetric in k, j):                          */
/*   dL/dx_k = sum_{j != k} K_kj (m_k ga_j - m_j ga_k)                        */
/*           - sum_{j != k} d (m_k gp_j + m_j gp_k) / s^3                     */
/*   dL/dm_k = - sum_{j != k} ga_j . d / s^3 - sum_{j != k} gp_j / s          */
/* gp, gm may be NULL (gp NULL means no potential cotangent).                 */
/* ------------------------------------------------------------------------- */
OR_EXPORT void oracle_vjp(int64_t n, const double *x, const double *m, double eps,
                          const double *ga, const double *gp, double *gx, double *gm)
{
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t k = 0; k < n; ++k) {
        double rx = 0.0, ry = 0.0, rz = 0.0, rm = 0.0;
        const double gpk = gp ? gp[k] : 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == k)
                continue;
            const double dx = x[3 * j + 0] - x[3 * k + 0];
            const double dy = x[3 * j + 1] - x[3 * k + 1];
            const double dz = x[3 * j + 2] - x[3 * k + 2];
            const double s2 = dx * dx + dy * dy + dz * dz + eps2;
            const double s = sqrt(s2);
            const double s3 = s2 * s;
            const double s5 = s3 * s2;
            const double wx = m[k] * ga[3 * j + 0] - m[j] * ga[3 * k + 0];
            const double wy = m[k] * ga[3 * j + 1] - m[j] * ga[3 * k + 1];
            const double wz = m[k] * ga[3 * j + 2] - m[j] * ga[3 * k + 2];
            const double dw = dx * wx + dy * wy + dz * wz;
            rx += wx / s3 - 3.0 * dx * dw / s5;
            ry += wy / s3 - 3.0 * dy * dw / s5;
            rz += wz / s3 - 3.0 * dz * dw / s5;
            const double gpj = gp ? gp[j] : 0.0;
            const double q = m[k] * gpj + m[j] * gpk;
            rx -= dx * q / s3;
            ry -= dy * q / s3;
            rz -= dz * q / s3;
            const double gd = ga[3 * j + 0] * dx + ga[3 * j + 1] * dy + ga[3 * j + 2] * dz;
            rm -= gd / s3 + gpj / s;
        }
        gx[3 * k + 0] = rx;
        gx[3 * k + 1] = ry;
        gx[3 * k + 2] = rz;
        if (gm)
            gm[k] = rm;
    }
}

/* ------------------------------------------------------------------------- */
/* Kick-drift-kick leapfrog in FP64 (the paper has no integrator; this is the */
/* standard second-order symplectic scheme):                                  */
/*   v_half = v + (dt/2) a(x);  x' = x + dt v_half;  v' = v_half + (dt/2) a(x') */
/* a(x) is evaluated once per distinct x.  x, v are updated in place.  If     */
/* traj is not NULL it receives x_0 .. x_nsteps ((nsteps+1) * n * 3).  acc    */
/* receives a(x_nsteps) if not NULL.                                          */
/* ------------------------------------------------------------------------- */
OR_EXPORT void oracle_rollout(int64_t n, double *x, double *v, const double *m, double eps,
                              double dt, int64_t nsteps, double *traj, double *acc_out)
{
    const size_t n3 = 3 * (size_t)n;
    double *a = (double *)malloc(sizeof(double) * (n3 ? n3 : 1));
    oracle_force_all(n, x, m, eps, a, NULL);
    if (traj)
        memcpy(traj, x, n3 * sizeof(double));
    for (int64_t t = 0; t < nsteps; ++t) {
        for (size_t q = 0; q < n3; ++q)
            v[q] += 0.5 * dt * a[q];
        for (size_t q = 0; q < n3; ++q)
            x[q] += dt * v[q];
        oracle_force_all(n, x, m, eps, a, NULL);
        for (size_t q = 0; q < n3; ++q)
            v[q] += 0.5 * dt * a[q];
        if (traj)
            memcpy(traj + (size_t)(t + 1) * n3, x, n3 * sizeof(double));
    }
    if (acc_out)
        memcpy(acc_out, a, n3 * sizeof(double));
    free(a);
}

/* ------------------------------------------------------------------------- */
/* Reverse mode through nsteps KDK steps whose positions x_0 .. x_nsteps are  */
/* stored in traj.  On entry xb, vb hold dL/dx_T, dL/dv_T; on exit dL/dx_0,   */
/* dL/dv_0; dL/dm is added to mb.  Reverse of one step (x_t, v_t) ->          */
/* (x_{t+1}, v_{t+1}), h = dt/2:                                              */
/*   abar_{t+1} += h vbar_{t+1}          (second kick used a(x_{t+1}))         */
/*   xbar_{t+1} += VJP_x(x_{t+1}, abar_{t+1}); mbar += VJP_m(...)             */
/*   vbar_half   = vbar_{t+1} + dt xbar_{t+1}                                 */
/*   xbar_t      = xbar_{t+1};  vbar_t = vbar_half                            */
/*   abar_t      = h vbar_half           (first kick used a(x_t))             */
/* and finally xbar_0 += VJP_x(x_0, abar_0).  The two kicks that use a(x_t)   */
/* have their cotangents summed before one VJP, as a(x_t) is one evaluation.  */
/* With nsteps = 0 abar_0 = 0: the map is the identity.                       */
/* ------------------------------------------------------------------------- */
static void reverse_kdk(int64_t n, const double *traj, const double *m, double eps, double dt,
                        int64_t nsteps, double *xb, double *vb, double *mb)
{
    const size_t n3 = 3 * (size_t)n;
    const size_t nn = n3 ? n3 : 1;
    double *ab = (double *)calloc(nn, sizeof(double));
    double *tx = (double *)malloc(sizeof(double) * nn);
    double *tm = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    const double h = 0.5 * dt;
    for (int64_t t = nsteps - 1; t >= 0; --t) {
        const double *x1 = traj + (size_t)(t + 1) * n3;
        for (size_t q = 0; q < n3; ++q)
            ab[q] += h * vb[q];
        oracle_vjp(n, x1, m, eps, ab, NULL, tx, tm);
        for (size_t q = 0; q < n3; ++q)
            xb[q] += tx[q];
        for (int64_t i = 0; i < n; ++i)
            mb[i] += tm[i];
        for (size_t q = 0; q < n3; ++q) {
            vb[q] += dt * xb[q];
            ab[q] = h * vb[q];
        }
    }
    oracle_vjp(n, traj, m, eps, ab, NULL, tx, tm);
    for (size_t q = 0; q < n3; ++q)
        xb[q] += tx[q];
    for (int64_t i = 0; i < n; ++i)
        mb[i] += tm[i];
    free(ab); free(tx); free(tm);
}

/* ------------------------------------------------------------------------- */
/* Loss L = (1/n) sum_i |x_i(T) - y_i|^2 after nsteps KDK steps from (x0, v0), */
/* and its gradient with respect to x0, v0 and m by reverse mode through the  */
/* KDK map (reverse_kdk with dL/dx_T = 2 (x_T - y) / n, dL/dv_T = 0).         */
/* gx0, gv0, gm may each be NULL.  Returns L.                                 */
/* ------------------------------------------------------------------------- */
OR_EXPORT double oracle_rollout_loss_grad(int64_t n, const double *x0, const double *v0,
                                          const double *m, double eps, double dt,
                                          int64_t nsteps, const double *y,
                                          double *gx0, double *gv0, double *gm)
{
    const size_t n3 = 3 * (size_t)n;
    const size_t nn = n3 ? n3 : 1;
    double *traj = (double *)malloc(sizeof(double) * nn * (size_t)(nsteps + 1));
    double *x = (double *)malloc(sizeof(double) * nn);
    double *v = (double *)malloc(sizeof(double) * nn);
    memcpy(x, x0, n3 * sizeof(double));
    memcpy(v, v0, n3 * sizeof(double));
    oracle_rollout(n, x, v, m, eps, dt, nsteps, traj, NULL);

    double loss = 0.0;
    const double *xT = traj + (size_t)nsteps * n3;
    for (size_t q = 0; q < n3; ++q)
        loss += (xT[q] - y[q]) * (xT[q] - y[q]);
    loss /= (double)(n > 0 ? n : 1);

    double *xb = (double *)calloc(nn, sizeof(double));
    double *vb = (double *)calloc(nn, sizeof(double));
    double *mb = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (size_t q = 0; q < n3; ++q)
        xb[q] = 2.0 * (xT[q] - y[q]) / (double)n;
    reverse_kdk(n, traj, m, eps, dt, nsteps, xb, vb, mb);

    if (gx0)
        memcpy(gx0, xb, n3 * sizeof(double));
    if (gv0)
        memcpy(gv0, vb, n3 * sizeof(double));
    if (gm)
        memcpy(gm, mb, (size_t)n * sizeof(double));
    free(traj); free(x); free(v); free(xb); free(vb); free(mb);
    return loss;
}

/* ------------------------------------------------------------------------- */
/* Vector-Jacobian product of the whole rollout for any cotangents of the     */
/* final state: given xbT = dL/dx_T and vbT = dL/dv_T (either NULL for zero),  */
/* writes dL/dx0, dL/dv0 and dL/dm (each may be NULL).                        */
/* ------------------------------------------------------------------------- */
OR_EXPORT void oracle_rollout_vjp(int64_t n, const double *x0, const double *v0, const double *m,
                                  double eps, double dt, int64_t nsteps, const double *xbT,
                                  const double *vbT, double *gx0, double *gv0, double *gm)
{
    const size_t n3 = 3 * (size_t)n;
    const size_t nn = n3 ? n3 : 1;
    double *traj = (double *)malloc(sizeof(double) * nn * (size_t)(nsteps + 1));
    double *x = (double *)malloc(sizeof(double) * nn);
    double *v = (double *)malloc(sizeof(double) * nn);
    memcpy(x, x0, n3 * sizeof(double));
    memcpy(v, v0, n3 * sizeof(double));
    oracle_rollout(n, x, v, m, eps, dt, nsteps, traj, NULL);
    double *xb = (double *)calloc(nn, sizeof(double));
    double *vb = (double *)calloc(nn, sizeof(double));
    double *mb = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    if (xbT)
        memcpy(xb, xbT, n3 * sizeof(double));
    if (vbT)
        memcpy(vb, vbT, n3 * sizeof(double));
    reverse_kdk(n, traj, m, eps, dt, nsteps, xb, vb, mb);
    if (gx0)
        memcpy(gx0, xb, n3 * sizeof(double));
    if (gv0)
        memcpy(gv0, vb, n3 * sizeof(double));
    if (gm)
        memcpy(gm, mb, (size_t)n * sizeof(double));
    free(traj); free(x); free(v); free(xb); free(vb); free(mb);
}

/* ------------------------------------------------------------------------- */
/* Single-precision replay of the paper's two accumulation orders, used only  */
/* to compare error magnitudes with the paper's Table 2 (Sec. 3.4).           */
/* Pair term in FP32 with IEEE 1/sqrt: r2 = (dx^2 + dy^2) + (dz^2 + eps2),    */
/* w = m_j (1/sqrt(r2))^3, term = w d.  The i-set equals the j-set and the    */
/* self pair is included (its term is exactly zero), as in the paper's test.  */
/*   nbag == 0: "DIRECT" - one FP32 accumulator over j = 0 .. n-1.            */
/*   nbag  > 0: Chamomile FORCE-LOOP, eq. (2) - an FP32 partial over each     */
/*              consecutive bag of nbag j's, added to an FP32 running force.  */
/* Results for the listed i (idx[0..k)) are returned widened to double.       */
/* This translation unit is compiled without FMA contraction.                 */
/* ------------------------------------------------------------------------- */
OR_EXPORT void oracle_fp32_replay(int64_t n, const float *x, const float *m, float eps2,
                                  int64_t nbag, int64_t k, const int64_t *idx, double *acc)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < k; ++t) {
        const int64_t i = idx[t];
        const float xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
        float tot[3] = {0.0f, 0.0f, 0.0f};
        float part[3] = {0.0f, 0.0f, 0.0f};
        const int64_t bag = nbag > 0 ? nbag : n;
        for (int64_t j0 = 0; j0 < n; j0 += bag) {
            const int64_t j1 = (j0 + bag < n) ? j0 + bag : n;
            float *dst = nbag > 0 ? part : tot;
            if (nbag > 0)
                part[0] = part[1] = part[2] = 0.0f;
            for (int64_t j = j0; j < j1; ++j) {
                const float dx = x[3 * j] - xi;
                const float dy = x[3 * j + 1] - yi;
                const float dz = x[3 * j + 2] - zi;
                const float r2 = (dx * dx + dy * dy) + (dz * dz + eps2);
                const float rinv = 1.0f / sqrtf(r2);
                const float w = m[j] * (rinv * rinv * rinv);
                dst[0] += w * dx;
                dst[1] += w * dy;
                dst[2] += w * dz;
            }
            if (nbag > 0) {
                tot[0] += part[0];
                tot[1] += part[1];
                tot[2] += part[2];
            }
        }
        acc[3 * t + 0] = tot[0];
        acc[3 * t + 1] = tot[1];
        acc[3 * t + 2] = tot[2];
    }
}

/* ------------------------------------------------------------------------- */
/* Fourth-order Hermite integration with a shared step (the integrator the     */
/* paper's force-jerk interaction serves, Sec. 4.1), in the predictor-         */
/* evaluate-corrector form of Makino & Aarseth (1992):                          */
/*   x_p = x + v dt + a dt^2/2 + j dt^3/6,   v_p = v + a dt + j dt^2/2          */
/*   (a1, j1) = F(x_p, v_p)                                                     */
/*   v' = v + (a + a1) dt/2 + (j - j1) dt^2/12                                  */
/*   x' = x + (v + v') dt/2 + (a - a1) dt^2/12                                  */
/* and (a, j) <- (a1, j1) for the next step.  (a, j) at the start are computed  */
/* from (x, v).  x, v are updated in place; acc_out, jerk_out (may be NULL)     */
/* receive the last (a1, j1).                                                   */
/* ------------------------------------------------------------------------- */
OR_EXPORT void oracle_hermite(int64_t n, double *x, double *v, const double *m, double eps,
                              double dt, int64_t nsteps, double *acc_out, double *jerk_out)
{
    const size_t n3 = 3 * (size_t)n;
    const size_t bytes = sizeof(double) * (n3 ? n3 : 1);
    double *a = (double *)malloc(bytes), *j = (double *)malloc(bytes);
    double *a1 = (double *)malloc(bytes), *j1 = (double *)malloc(bytes);
    double *xp = (double *)malloc(bytes), *vp = (double *)malloc(bytes);
    int64_t *self = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i)
        self[i] = i;
    oracle_force_jerk(n, x, v, m, n, x, v, self, eps, a, j, NULL);
    for (int64_t t = 0; t < nsteps; ++t) {
        for (size_t q = 0; q < n3; ++q) {
            xp[q] = x[q] + v[q] * dt + a[q] * dt * dt / 2.0 + j[q] * dt * dt * dt / 6.0;
            vp[q] = v[q] + a[q] * dt + j[q] * dt * dt / 2.0;
        }
        oracle_force_jerk(n, xp, vp, m, n, xp, vp, self, eps, a1, j1, NULL);
        for (size_t q = 0; q < n3; ++q) {
            const double vn = v[q] + (a[q] + a1[q]) * dt / 2.0 + (j[q] - j1[q]) * dt * dt / 12.0;
            x[q] = x[q] + (v[q] + vn) * dt / 2.0 + (a[q] - a1[q]) * dt * dt / 12.0;
            v[q] = vn;
            a[q] = a1[q];
            j[q] = j1[q];
        }
    }
    if (acc_out)
        memcpy(acc_out, a, n3 * sizeof(double));
    if (jerk_out)
        memcpy(jerk_out, j, n3 * sizeof(double));
    free(a); free(j); free(a1); free(j1); free(xp); free(vp); free(self);
}

/* Number of OpenMP threads the oracle uses (1 without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
OR_EXPORT int oracle_threads(void) { return omp_get_max_threads(); }
OR_EXPORT void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
#else
OR_EXPORT int oracle_threads(void) { return 1; }
OR_EXPORT void oracle_set_threads(int n) { (void)n; }
#endif
