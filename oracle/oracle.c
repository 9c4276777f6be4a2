/*
 * FP64 CPU oracle for the all-pairs softened-gravity N-body hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. The GPU product path
 * never calls it and shares no code with it.
 *
 * Every routine is the plain definition written out in double precision:
 * i runs over particles (OpenMP-parallel; each i is independent), and each
 * per-particle sum runs over j in ascending order with j == i skipped, so the
 * result does not depend on the thread count.
 *
 * Physics. The paper's N-body miniapp (Sec. II-A, Sec. V-B) computes the
 * force between every pair of particles, N_p^2 operations per evaluation, and
 * advances positions with a Verlet half-step scheme; its total energy is a
 * reduction over all particles fused into the force pass (Sec. VI). The pair
 * law used here is Plummer-softened Newtonian gravity in place of the paper's
 * Lennard-Jones Eq. (1):
 *     d_ij  = x_j - x_i,   s_ij = |d_ij|^2 + eps^2
 *     a_i   =  G sum_{j != i} m_j d_ij s_ij^{-3/2}
 *     phi_i = -G sum_{j != i} m_j s_ij^{-1/2}
 * The Verlet half-step scheme is read as kick-drift-kick leapfrog with force
 * reuse (one force evaluation per step plus one initial evaluation).
 * The paper's own Lennard-Jones law (Eq. (1)) and its boundary check (read as
 * reflective walls) are at the end of this file (oracle_lj_*).
 *
 * Layout: positions, velocities, accelerations are SoA planes [3][n]
 * (x plane, y plane, z plane), all double, host memory owned by the caller.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define EXPORT __attribute__((visibility("default")))

/* Sums of one particle i against all j in [0, n), j != i, in ascending j:
 * out = {sum m_j dx s^{-3/2}, sum m_j dy s^{-3/2}, sum m_j dz s^{-3/2}, -sum m_j s^{-1/2}}. */
static void force_at(int64_t n, const double *pos, const double *mass, double eps2, int64_t i, double out[4])
{
    const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double dx = X[j] - X[i];
        double dy = Y[j] - Y[i];
        double dz = Z[j] - Z[i];
        double s = dx * dx + dy * dy + dz * dz + eps2;
        double inv_r = 1.0 / sqrt(s);          /* s^{-1/2} */
        double inv_r3 = inv_r / s;             /* s^{-3/2} */
        ax += mass[j] * dx * inv_r3;
        ay += mass[j] * dy * inv_r3;
        az += mass[j] * dz * inv_r3;
        ph -= mass[j] * inv_r;
    }
    out[0] = ax; out[1] = ay; out[2] = az; out[3] = ph;
}

/* a_i and phi_i for i in [i0, i1) against all j in [0, n), j != i.
 * acc: [3][n] (only rows i0..i1-1 written), pot: [n] or NULL. */
static void forces_range(int64_t n, const double *pos, const double *mass, double G, double eps,
                         int64_t i0, int64_t i1, double *acc, double *pot)
{
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = i0; i < i1; ++i) {
        double r[4];
        force_at(n, pos, mass, eps2, i, r);
        acc[i] = G * r[0];
        acc[n + i] = G * r[1];
        acc[2 * n + i] = G * r[2];
        if (pot) pot[i] = G * r[3];
    }
}

/* All-pairs acceleration and (optionally) potential, definition as above. */
EXPORT void oracle_forces(int64_t n, const double *pos, const double *mass, double G, double eps,
                          double *acc, double *pot)
{
    forces_range(n, pos, mass, G, eps, 0, n, acc, pot);
}

/* Acceleration/potential of a chosen subset of particles against all j: the same
 * per-particle sums as oracle_forces (force_at), so each sampled row equals the full
 * call's row bitwise. idx[k] names particle i; output rows are packed:
 * acc_out [3][nidx], pot_out [nidx] (nullable). */
EXPORT void oracle_forces_sample(int64_t n, const double *pos, const double *mass, double G, double eps,
                                 int64_t nidx, const int64_t *idx, double *acc_out, double *pot_out)
{
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < nidx; ++k) {
        double r[4];
        force_at(n, pos, mass, eps2, idx[k], r);
        acc_out[k] = G * r[0];
        acc_out[nidx + k] = G * r[1];
        acc_out[2 * nidx + k] = G * r[2];
        if (pot_out) pot_out[k] = G * r[3];
    }
}

/* Energy and linear momentum of one system:
 *   KE = 1/2 sum_i m_i |v_i|^2,  PE = 1/2 sum_i m_i phi_i,  P = sum_i m_i v_i.
 * out[5] = {KE, PE, Px, Py, Pz}. phi is computed from its definition. */
EXPORT void oracle_energy_momentum(int64_t n, const double *pos, const double *vel, const double *mass,
                                   double G, double eps, double *out)
{
    double *pot = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *acc = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? 3 * n : 1));
    forces_range(n, pos, mass, G, eps, 0, n, acc, pot);
    double ke = 0.0, pe = 0.0, px = 0.0, py = 0.0, pz = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double vx = vel[i], vy = vel[n + i], vz = vel[2 * n + i];
        ke += 0.5 * mass[i] * (vx * vx + vy * vy + vz * vz);
        pe += 0.5 * mass[i] * pot[i];
        px += mass[i] * vx;
        py += mass[i] * vy;
        pz += mass[i] * vz;
    }
    out[0] = ke; out[1] = pe; out[2] = px; out[3] = py; out[4] = pz;
    free(pot);
    free(acc);
}

/* Kick-drift-kick leapfrog, `steps` steps of size dt, state updated in place.
 *   a = a(x)
 *   repeat: v += (dt/2) a;  x += dt v;  a = a(x);  v += (dt/2) a
 * traj (nullable): positions after every step, [steps+1][3][n], traj[0] = x_0.
 * energy (nullable): [steps+1][5] = energy/momentum at every integer step. */
EXPORT void oracle_kdk(int64_t n, double G, double eps, double dt, int64_t steps,
                       double *pos, double *vel, const double *mass, double *traj, double *energy)
{
    double *acc = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? 3 * n : 1));
    forces_range(n, pos, mass, G, eps, 0, n, acc, NULL);
    if (traj) memcpy(traj, pos, sizeof(double) * (size_t)(3 * n));
    if (energy) oracle_energy_momentum(n, pos, vel, mass, G, eps, energy);
    const double h = dt, hh = 0.5 * dt;
    for (int64_t step = 0; step < steps; ++step) {
        for (int64_t k = 0; k < 3 * n; ++k) vel[k] += hh * acc[k];
        for (int64_t k = 0; k < 3 * n; ++k) pos[k] += h * vel[k];
        forces_range(n, pos, mass, G, eps, 0, n, acc, NULL);
        for (int64_t k = 0; k < 3 * n; ++k) vel[k] += hh * acc[k];
        if (traj) memcpy(traj + (size_t)(step + 1) * 3 * n, pos, sizeof(double) * (size_t)(3 * n));
        if (energy) oracle_energy_momentum(n, pos, vel, mass, G, eps, energy + 5 * (step + 1));
    }
    free(acc);
}

/* Vector-Jacobian product of the acceleration map (x, m) -> a.
 * Given a cotangent lam [3][n] on a, returns the gradient of sum_i lam_i . a_i:
 *   gx_k = G sum_{j != k} T(d_kj) (m_k lam_j - m_j lam_k),
 *   gm_k = -G sum_{j != k} s_kj^{-3/2} d_kj . lam_j,
 * with d_kj = x_j - x_k, s_kj = |d_kj|^2 + eps^2 and the softened tidal tensor
 *   T(d) = s^{-3/2} I - 3 s^{-5/2} d d^T  (the Jacobian of d s^{-3/2} w.r.t. d).
 * vjp_at: the unscaled sums of particle k, ascending j, out = {gx, gy, gz, gm}. */
static void vjp_at(int64_t n, const double *pos, const double *mass, double eps2, const double *lam, int64_t k,
                   double out[4])
{
    const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
    const double *LX = lam, *LY = lam + n, *LZ = lam + 2 * n;
    double gxx = 0.0, gxy = 0.0, gxz = 0.0, gmk = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == k) continue;
        double dx = X[j] - X[k], dy = Y[j] - Y[k], dz = Z[j] - Z[k];
        double s = dx * dx + dy * dy + dz * dz + eps2;
        double inv_r = 1.0 / sqrt(s);
        double s_m32 = inv_r / s;             /* s^{-3/2} */
        double s_m52 = s_m32 / s;             /* s^{-5/2} */
        /* u = m_k lam_j - m_j lam_k */
        double ux = mass[k] * LX[j] - mass[j] * LX[k];
        double uy = mass[k] * LY[j] - mass[j] * LY[k];
        double uz = mass[k] * LZ[j] - mass[j] * LZ[k];
        /* T(d) u = s^{-3/2} u - 3 s^{-5/2} d (d . u) */
        double du = dx * ux + dy * uy + dz * uz;
        gxx += s_m32 * ux - 3.0 * s_m52 * dx * du;
        gxy += s_m32 * uy - 3.0 * s_m52 * dy * du;
        gxz += s_m32 * uz - 3.0 * s_m52 * dz * du;
        double dl = dx * LX[j] + dy * LY[j] + dz * LZ[j];
        gmk -= s_m32 * dl;
    }
    out[0] = gxx; out[1] = gxy; out[2] = gxz; out[3] = gmk;
}

/* The full VJP: the results are ADDED into gx [3][n] and gm [n]. */
EXPORT void oracle_force_vjp(int64_t n, const double *pos, const double *mass, double G, double eps,
                             const double *lam, double *gx, double *gm)
{
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n; ++k) {
        double r[4];
        vjp_at(n, pos, mass, eps2, lam, k, r);
        gx[k] += G * r[0];
        gx[n + k] += G * r[1];
        gx[2 * n + k] += G * r[2];
        gm[k] += G * r[3];
    }
}

/* The VJP's rows of the particles idx[0 .. nidx-1] only (the same per-particle sums as
 * oracle_force_vjp, so each row equals the full call's bitwise when gx, gm start at 0);
 * written (not added) packed: gx_out [3][nidx], gm_out [nidx]. */
EXPORT void oracle_force_vjp_sample(int64_t n, const double *pos, const double *mass, double G, double eps,
                                    const double *lam, int64_t nidx, const int64_t *idx, double *gx_out,
                                    double *gm_out)
{
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < nidx; ++k) {
        double r[4];
        vjp_at(n, pos, mass, eps2, lam, idx[k], r);
        gx_out[k] = 0.0 + G * r[0];
        gx_out[nidx + k] = 0.0 + G * r[1];
        gx_out[2 * nidx + k] = 0.0 + G * r[2];
        gm_out[k] = 0.0 + G * r[3];
    }
}

/* Gradient of a scalar function of the final state of a K-step KDK rollout
 * with respect to the initial positions, velocities and the masses
 * (discretise-then-differentiate: the exact adjoint of the discrete map).
 *
 * Inputs: the initial state (pos0, vel0, mass) and the cotangents of the final
 * state gpos_K = dL/dx_K, gvel_K = dL/dv_K. Outputs gpos0, gvel0 [3][n], gmass [n].
 *
 * Reverse sweep of the step  v' = v + h/2 a(x); x+ = x + h v'; v+ = v' + h/2 a(x+):
 *   gx = gpos_K, gv = gvel_K, gm = 0
 *   (gx, gm) += VJP(x_K, h/2 gv)                    second half-kick of the last step
 *   for n = K-1 down to 0:
 *       gv += h gx                                   drift
 *       (gx, gm) += VJP(x_n, w gv), w = h (n > 0), h/2 (n = 0)
 * The two half-kicks that meet at x_n (second of step n-1, first of step n)
 * read the same velocity cotangent, so they merge into one VJP of weight h.
 * The forward trajectory x_0..x_K is stored in full (no checkpointing). */
EXPORT void oracle_rollout_adjoint(int64_t n, double G, double eps, double dt, int64_t steps,
                                   const double *pos0, const double *vel0, const double *mass,
                                   const double *gpos_K, const double *gvel_K,
                                   double *gpos0, double *gvel0, double *gmass)
{
    const size_t plane = (size_t)(3 * n);
    double *traj = (double *)malloc(sizeof(double) * plane * (size_t)(steps + 1) + 8);
    double *x = (double *)malloc(sizeof(double) * plane + 8);
    double *v = (double *)malloc(sizeof(double) * plane + 8);
    double *lam = (double *)malloc(sizeof(double) * plane + 8);
    memcpy(x, pos0, sizeof(double) * plane);
    memcpy(v, vel0, sizeof(double) * plane);
    oracle_kdk(n, G, eps, dt, steps, x, v, mass, traj, NULL);

    const double h = dt;
    memcpy(gpos0, gpos_K, sizeof(double) * plane);
    memcpy(gvel0, gvel_K, sizeof(double) * plane);
    for (int64_t i = 0; i < n; ++i) gmass[i] = 0.0;

    for (size_t k = 0; k < plane; ++k) lam[k] = 0.5 * h * gvel0[k];
    oracle_force_vjp(n, traj + (size_t)steps * plane, mass, G, eps, lam, gpos0, gmass);
    for (int64_t s = steps - 1; s >= 0; --s) {
        for (size_t k = 0; k < plane; ++k) gvel0[k] += h * gpos0[k];
        const double w = (s > 0) ? h : 0.5 * h;
        for (size_t k = 0; k < plane; ++k) lam[k] = w * gvel0[k];
        oracle_force_vjp(n, traj + (size_t)s * plane, mass, G, eps, lam, gpos0, gmass);
    }
    free(traj); free(x); free(v); free(lam);
}

/* Mean squared distance of the final positions to a target set,
 *   L = (1/n) sum_i |x_i - y_i|^2,
 * and its gradient with respect to x: dL/dx_i = 2 (x_i - y_i) / n (grad nullable). */
EXPORT double oracle_loss_msd(int64_t n, const double *pos, const double *target, double *grad)
{
    double acc = 0.0;
    for (int64_t c = 0; c < 3; ++c)
        for (int64_t i = 0; i < n; ++i) {
            double d = pos[c * n + i] - target[c * n + i];
            acc += d * d;
            if (grad) grad[c * n + i] = 2.0 * d / (double)n;
        }
    return n > 0 ? acc / (double)n : 0.0;
}

/* Thread count of later parallel regions (t >= 1); the results do not depend on it. */
EXPORT void oracle_set_threads(int t)
{
#ifdef _OPENMP
    if (t >= 1) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

EXPORT int oracle_num_threads(void)
{
    int t = 1;
#ifdef _OPENMP
#pragma omp parallel
    {
#pragma omp single
        t = omp_get_num_threads();
    }
#endif
    return t;
}

/* ---------------------------------------------------------------------------
 * Lennard-Jones gas: the paper's pair law, Eq. (1), V(r) = 4 e [(s/r)^12 - (s/r)^6]
 * with F = -grad V = 24 e [2 s^12 / r^13 - s^6 / r^7] r_hat (repulsive for r < 2^{1/6} s).
 * An optional softening w enters as r^2 -> r^2 + w^2 (w = 0 is the plain law).
 * Acceleration a_i = F_i / m_i. The per-particle potential is returned per unit mass,
 * pot_i = (1/m_i) sum_{j != i} V(r_ij), so that PE = 1/2 sum_i m_i pot_i = sum_{i<j} V(r_ij)
 * (the same bookkeeping as the gravitational phi).
 * --------------------------------------------------------------------------- */
EXPORT void oracle_lj_forces(int64_t n, const double *pos, const double *mass, double sigma, double epsilon,
                             double soft, double *acc, double *pot)
{
    const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double fx = 0.0, fy = 0.0, fz = 0.0, v = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            /* separation from j to i: the force on i points along x_i - x_j when repulsive */
            double rx = X[i] - X[j], ry = Y[i] - Y[j], rz = Z[i] - Z[j];
            double r2 = rx * rx + ry * ry + rz * rz + soft * soft;
            double sr2 = sigma * sigma / r2;
            double sr6 = sr2 * sr2 * sr2;
            double sr12 = sr6 * sr6;
            /* |F| / r = 24 e (2 (s/r)^12 - (s/r)^6) / r^2 */
            double f_over_r = 24.0 * epsilon * (2.0 * sr12 - sr6) / r2;
            fx += f_over_r * rx;
            fy += f_over_r * ry;
            fz += f_over_r * rz;
            v += 4.0 * epsilon * (sr12 - sr6);
        }
        acc[i] = fx / mass[i];
        acc[n + i] = fy / mass[i];
        acc[2 * n + i] = fz / mass[i];
        if (pot) pot[i] = v / mass[i];
    }
}

/* Reflective walls of the box [lo, hi]^3 (the paper's boundary check): a particle
 * past a wall is mirrored back into the box and its velocity component flips. */
static void reflect(int64_t n, double *pos, double *vel, const double *lo, const double *hi)
{
    for (int c = 0; c < 3; ++c)
        for (int64_t i = 0; i < n; ++i) {
            double x = pos[c * n + i];
            if (x < lo[c]) {
                pos[c * n + i] = 2.0 * lo[c] - x;
                vel[c * n + i] = -vel[c * n + i];
            } else if (x > hi[c]) {
                pos[c * n + i] = 2.0 * hi[c] - x;
                vel[c * n + i] = -vel[c * n + i];
            }
        }
}

/* Lennard-Jones energy of one system: out = {KE, PE, Px, Py, Pz}. */
EXPORT void oracle_lj_energy(int64_t n, const double *pos, const double *vel, const double *mass, double sigma,
                             double epsilon, double soft, double *out)
{
    double *pot = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *acc = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? 3 * n : 1));
    oracle_lj_forces(n, pos, mass, sigma, epsilon, soft, acc, pot);
    double ke = 0.0, pe = 0.0, px = 0.0, py = 0.0, pz = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double vx = vel[i], vy = vel[n + i], vz = vel[2 * n + i];
        ke += 0.5 * mass[i] * (vx * vx + vy * vy + vz * vz);
        pe += 0.5 * mass[i] * pot[i];
        px += mass[i] * vx;
        py += mass[i] * vy;
        pz += mass[i] * vz;
    }
    out[0] = ke; out[1] = pe; out[2] = px; out[3] = py; out[4] = pz;
    free(pot);
    free(acc);
}

/* Kick-drift-kick steps of the Lennard-Jones gas with the reflective-wall check after
 * every drift (box given by lo[3], hi[3]; box == NULL: open space). energy nullable,
 * [steps+1][5]. */
EXPORT void oracle_lj_kdk(int64_t n, double sigma, double epsilon, double soft, double dt, int64_t steps,
                          double *pos, double *vel, const double *mass, const double *lo, const double *hi,
                          double *energy)
{
    double *acc = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? 3 * n : 1));
    oracle_lj_forces(n, pos, mass, sigma, epsilon, soft, acc, NULL);
    if (energy) oracle_lj_energy(n, pos, vel, mass, sigma, epsilon, soft, energy);
    const double h = dt, hh = 0.5 * dt;
    for (int64_t step = 0; step < steps; ++step) {
        for (int64_t k = 0; k < 3 * n; ++k) vel[k] += hh * acc[k];
        for (int64_t k = 0; k < 3 * n; ++k) pos[k] += h * vel[k];
        if (lo && hi) reflect(n, pos, vel, lo, hi);
        oracle_lj_forces(n, pos, mass, sigma, epsilon, soft, acc, NULL);
        for (int64_t k = 0; k < 3 * n; ++k) vel[k] += hh * acc[k];
        if (energy) oracle_lj_energy(n, pos, vel, mass, sigma, epsilon, soft, energy + 5 * (step + 1));
    }
    free(acc);
}

/* ---------------------------------------------------------------------------
 * Diagnostics of one system from its state and a force evaluation (any pair law):
 *   out = {KE, PE, Px, Py, Pz, Lx, Ly, Lz, W, M}
 *   KE = 1/2 sum m |v|^2, PE = 1/2 sum m pot, P = sum m v, L = sum m x cross v,
 *   W = sum m x . a (the virial of the pair forces), M = sum m.
 * pot is the per-particle potential per unit mass and acc the acceleration, as the
 * force routines return them.
 * --------------------------------------------------------------------------- */
EXPORT void oracle_diagnostics(int64_t n, const double *pos, const double *vel, const double *mass,
                               const double *pot, const double *acc, double *out)
{
    for (int k = 0; k < 10; ++k) out[k] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double m = mass[i];
        const double x = pos[i], y = pos[n + i], z = pos[2 * n + i];
        const double vx = vel[i], vy = vel[n + i], vz = vel[2 * n + i];
        const double ax = acc[i], ay = acc[n + i], az = acc[2 * n + i];
        out[0] += 0.5 * m * (vx * vx + vy * vy + vz * vz);
        out[1] += 0.5 * m * pot[i];
        out[2] += m * vx;
        out[3] += m * vy;
        out[4] += m * vz;
        out[5] += m * (y * vz - z * vy);
        out[6] += m * (z * vx - x * vz);
        out[7] += m * (x * vy - y * vx);
        out[8] += m * (x * ax + y * ay + z * az);
        out[9] += m;
    }
}
