/*
 * FP64 CPU oracle for the cascaded (central-moment) lattice Boltzmann update
 * with symmetrized (Strang) operator-split force and source steps
 * (Hajabdollahi & Premnath, arXiv:1806.10247).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or generator with the GPU library.
 *
 * Every per-node formula below is written out from the paper:
 *   - D2Q9 flow: velocity set eq. (15); pre-collision half force step eq. (25);
 *     cascaded collision eq. (23); post-collision half force step as a change
 *     of the first-order moments eq. (31); post-collision populations eq. (32);
 *     pull form of the streaming step eq. (22b); algorithm steps (i)-(vi) of
 *     Sec. 4.
 *   - D2Q5 scalar: velocity set eq. (34); pre-collision half source step
 *     eq. (43); cascaded collision eq. (41); post-collision half source step
 *     as a change of the zeroth moment eq. (47); post-collision populations
 *     eq. (48).  The u^2*phi terms of eq. (41) are taken with a minus sign
 *     (the printed plus sign does not relax the second-order central moments
 *     of eq. (37) to the equilibria of eq. (39)); a flag evaluates the printed
 *     sign for the test that documents this reading.
 *   - D3Q27 flow: the paper only states (Appendix A) that its 3D derivation
 *     extends to D3Q27.  The oracle builds it by the lattice-independent
 *     construction that reproduces the printed D2Q9 update: relax the
 *     central moments about the half-forced velocity, computed from the raw
 *     moments of eq. (21)/(g8) with the first-order raw moments replaced by
 *     rho*u (as eq. (23) does), map the moment change back with the inverse
 *     raw-moment matrix, and add the post-collision kick F.e_alpha/<e_x|e_x>
 *     (eq. (31) has <e_x|e_x> = 6, eq. (13A) has 10; D3Q27 has 18).
 *     The same routine run on D2Q9 must equal eq. (23)/(31)/(32) exactly.
 *   - D3Q15 flow (Appendix A): velocities eq. (A1), basis eq. (2A), the
 *     cascaded collision eq. (6A), the half force steps eqs. (8A), (13A),
 *     f^p = f + K g.  Readings: the trace relaxes towards rho (eq. (6A) prints
 *     g_9 without it), the fourth-order equilibrium of g_14 is rho/9 (the
 *     paper leaves it undefined; it is the only value for which the rest
 *     state, whose k_xxyy is 8/72 = 1/9 with the isotropy-fixed weights, is a
 *     fixed point of the collision), and the post-collision rows are K g (the
 *     printed row 12 has the sign of g_13 flipped).
 *   - Time-dependent forcing: each half step uses the trapezoidal average of
 *     the force over that half step (Sec. 6, Womersley flow).
 *   - Walls: halfway bounce-back (Sec. 6, Poiseuille flow); moving walls,
 *     fixed-value scalar walls and the viscous-heating source of the thermal
 *     Couette problem (Sec. 6), whose wall treatment the paper leaves open.
 *
 * Compiled with gcc, no fast-math and no FP contraction, so that every
 * operation is one IEEE double rounding.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_D2Q9 0
#define ORC_D2Q9_D2Q5 1
#define ORC_D3Q27 2
#define ORC_D3Q15 3

#define ORC_PERIODIC 0
#define ORC_BOUNCE_BACK 1

#define ORC_TIME_CONSTANT 0
#define ORC_TIME_COS 1

/* ------------------------------------------------------------------------ */
/* Velocity sets                                                              */
/* ------------------------------------------------------------------------ */

/* D2Q9, eq. (15). */
static const int D2Q9_EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int D2Q9_EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* D2Q5, eq. (34). */
static const int D2Q5_EX[5] = {0, 1, 0, -1, 0};
static const int D2Q5_EY[5] = {0, 0, 1, 0, -1};

/* D3Q27 (not listed in the paper).  Direction alpha = d(ex) + 3 d(ey) + 9 d(ez)
 * with d(0) = 0, d(+1) = 1, d(-1) = 2. */
static int d3q27_component(int alpha, int axis) {
    int digit = alpha;
    for (int i = 0; i < axis; ++i) digit /= 3;
    digit %= 3;
    return digit == 0 ? 0 : (digit == 1 ? 1 : -1);
}

/* D3Q15, eq. (A1) (paper order). */
static const int D3Q15_EX[15] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
static const int D3Q15_EY[15] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
static const int D3Q15_EZ[15] = {0, 0, 0, 0, 0, 1, -1, 1, 1, 1, 1, -1, -1, -1, -1};

int orc_num_dirs(int lattice) { return lattice == ORC_D3Q27 ? 27 : (lattice == ORC_D3Q15 ? 15 : 9); }
int orc_num_dims(int lattice) { return lattice == ORC_D3Q27 || lattice == ORC_D3Q15 ? 3 : 2; }

/* Velocity component e_{alpha, axis} of the flow lattice. */
int orc_velocity(int lattice, int alpha, int axis) {
    if (lattice == ORC_D3Q27) return d3q27_component(alpha, axis);
    if (lattice == ORC_D3Q15) return axis == 0 ? D3Q15_EX[alpha] : (axis == 1 ? D3Q15_EY[alpha] : D3Q15_EZ[alpha]);
    if (axis == 0) return D2Q9_EX[alpha];
    if (axis == 1) return D2Q9_EY[alpha];
    return 0;
}

int orc_d2q5_velocity(int alpha, int axis) {
    if (axis == 0) return D2Q5_EX[alpha];
    if (axis == 1) return D2Q5_EY[alpha];
    return 0;
}

static int opposite_dir(int lattice, int alpha) {
    int q = orc_num_dirs(lattice), d = orc_num_dims(lattice);
    for (int b = 0; b < q; ++b) {
        int ok = 1;
        for (int i = 0; i < d; ++i)
            if (orc_velocity(lattice, b, i) != -orc_velocity(lattice, alpha, i)) ok = 0;
        if (ok) return b;
    }
    return -1;
}

static int d2q5_opposite(int alpha) {
    static const int opp[5] = {0, 3, 4, 1, 2};
    return opp[alpha];
}

/* ------------------------------------------------------------------------ */
/* D2Q9 cascaded collision with Strang forcing (Sec. 4)                       */
/* ------------------------------------------------------------------------ */

/* Post-collision populations, eq. (32): f^p = f + K g, rows as printed. */
void orc_d2q9_apply_k(const double f[9], const double g[9], double fp[9]) {
    fp[0] = f[0] + (g[0] - 4.0 * (g[3] - g[8]));
    fp[1] = f[1] + (g[0] + g[1] - g[3] + g[4] + 2.0 * (g[7] - g[8]));
    fp[2] = f[2] + (g[0] + g[2] - g[3] - g[4] + 2.0 * (g[6] - g[8]));
    fp[3] = f[3] + (g[0] - g[1] - g[3] + g[4] - 2.0 * (g[7] + g[8]));
    fp[4] = f[4] + (g[0] - g[2] - g[3] - g[4] - 2.0 * (g[6] + g[8]));
    fp[5] = f[5] + (g[0] + g[1] + g[2] + 2.0 * g[3] + g[5] - g[6] - g[7] + g[8]);
    fp[6] = f[6] + (g[0] - g[1] + g[2] + 2.0 * g[3] - g[5] - g[6] + g[7] + g[8]);
    fp[7] = f[7] + (g[0] - g[1] - g[2] + 2.0 * g[3] + g[5] + g[6] + g[7] + g[8]);
    fp[8] = f[8] + (g[0] + g[1] - g[2] + 2.0 * g[3] - g[5] + g[6] - g[7] + g[8]);
}

/*
 * One D2Q9 node: steps (i)-(iv) of Sec. 4 applied to the streamed populations.
 *   f      : streamed populations (input of step (i)), paper order
 *   fpre   : force averaged over the pre-collision half step
 *   ftot   : momentum change over the whole step (average of the two halves)
 *   omega  : omega_3 .. omega_8 of eq. (23)
 *   fp     : post-collision populations (output)
 *   u_out  : the half-forced velocity of eq. (25) (may be NULL)
 */
void orc_d2q9_collide(const double f[9], const double fpre[2], const double ftot[2],
                      const double omega[6], double fp[9], double u_out[2]) {
    /* Eq. (24): density and output momentum; eq. (21): raw moments. */
    double rho = 0, jx = 0, jy = 0, kxx = 0, kyy = 0, kxy = 0, kxxy = 0, kxyy = 0, kxxyy = 0;
    for (int a = 0; a < 9; ++a) {
        double ex = D2Q9_EX[a], ey = D2Q9_EY[a];
        rho += f[a];
        jx += f[a] * ex;
        jy += f[a] * ey;
        kxx += f[a] * ex * ex;
        kyy += f[a] * ey * ey;
        kxy += f[a] * ex * ey;
        kxxy += f[a] * ex * ex * ey;
        kxyy += f[a] * ex * ey * ey;
        kxxyy += f[a] * ex * ex * ey * ey;
    }
    /* Eq. (25): pre-collision half force step. */
    double ux = (jx + 0.5 * fpre[0]) / rho;
    double uy = (jy + 0.5 * fpre[1]) / rho;
    if (u_out) { u_out[0] = ux; u_out[1] = uy; }

    double w3 = omega[0], w4 = omega[1], w5 = omega[2], w6 = omega[3], w7 = omega[4], w8 = omega[5];
    double ux2 = ux * ux, uy2 = uy * uy;
    double g[9];
    /* Eq. (31): post-collision half force step as first-order moment change;
     * mass is a collision invariant. */
    g[0] = 0.0;
    g[1] = ftot[0] / 6.0;
    g[2] = ftot[1] / 6.0;
    /* Eq. (23): cascaded collision. */
    g[3] = w3 / 12.0 * ((2.0 / 3.0) * rho + rho * (ux2 + uy2) - (kxx + kyy));
    g[4] = w4 / 4.0 * (rho * (ux2 - uy2) - (kxx - kyy));
    g[5] = w5 / 4.0 * (rho * ux * uy - kxy);
    g[6] = w6 / 4.0 * (2.0 * rho * ux2 * uy + kxxy - 2.0 * ux * kxy - uy * kxx)
           - 0.5 * uy * (3.0 * g[3] + g[4]) - 2.0 * ux * g[5];
    g[7] = w7 / 4.0 * (2.0 * rho * ux * uy2 + kxyy - 2.0 * uy * kxy - ux * kyy)
           - 0.5 * ux * (3.0 * g[3] - g[4]) - 2.0 * uy * g[5];
    g[8] = w8 / 4.0 * ((1.0 / 9.0) * rho + 3.0 * rho * ux2 * uy2
                       - (kxxyy - 2.0 * ux * kxyy - 2.0 * uy * kxxy + ux2 * kyy + uy2 * kxx
                          + 4.0 * ux * uy * kxy))
           - 2.0 * g[3] - 0.5 * uy2 * (3.0 * g[3] + g[4]) - 0.5 * ux2 * (3.0 * g[3] - g[4])
           - 4.0 * ux * uy * g[5] - 2.0 * uy * g[6] - 2.0 * ux * g[7];
    /* Eq. (32). */
    orc_d2q9_apply_k(f, g, fp);
}

/* ------------------------------------------------------------------------ */
/* D2Q5 cascaded scalar collision with Strang source steps (Sec. 5)           */
/* ------------------------------------------------------------------------ */

/* Post-collision populations, eq. (48): g^p = g + L h, rows as printed. */
void orc_d2q5_apply_l(const double g[5], const double h[5], double gp[5]) {
    gp[0] = g[0] + (h[0] - 4.0 * h[3]);
    gp[1] = g[1] + (h[0] + h[1] + h[3] + h[4]);
    gp[2] = g[2] + (h[0] + h[2] + h[3] - h[4]);
    gp[3] = g[3] + (h[0] - h[1] + h[3] + h[4]);
    gp[4] = g[4] + (h[0] - h[2] + h[3] - h[4]);
}

/*
 * One D2Q5 node.
 *   g       : streamed scalar populations, paper order
 *   u       : fluid velocity at the node (the flow's half-forced velocity)
 *   spre    : source averaged over the pre-collision half step
 *   stot    : scalar change over the whole step
 *   omega   : omega^phi_1 .. omega^phi_4 of eq. (41)
 *   printed_sign : 1 evaluates eq. (41) with the printed "+(u_x^2 +- u_y^2) phi"
 *   gp      : post-collision populations (output)
 */
void orc_d2q5_collide(const double g[5], const double u[2], double spre, double stot,
                      const double omega[4], int printed_sign, double gp[5]) {
    /* Eq. (42) and eq. (38). */
    double phi0 = 0, kx = 0, ky = 0, kxx = 0, kyy = 0;
    for (int a = 0; a < 5; ++a) {
        double ex = D2Q5_EX[a], ey = D2Q5_EY[a];
        phi0 += g[a];
        kx += g[a] * ex;
        ky += g[a] * ey;
        kxx += g[a] * ex * ex;
        kyy += g[a] * ey * ey;
    }
    /* Eq. (43): pre-collision half source step. */
    double phi = phi0 + 0.5 * spre;
    double ux = u[0], uy = u[1];
    double cs2 = 1.0 / 3.0; /* c_{s phi}^2, Sec. 5 */
    double sgn = printed_sign ? 1.0 : -1.0;
    double h[5];
    /* Eq. (47): post-collision half source step as a zeroth-moment change. */
    h[0] = stot / 5.0;
    /* Eq. (41). */
    h[1] = omega[0] / 2.0 * (phi * ux - kx);
    h[2] = omega[1] / 2.0 * (phi * uy - ky);
    h[3] = omega[2] / 4.0 * (2.0 * cs2 * phi - (kxx + kyy) + 2.0 * (ux * kx + uy * ky)
                             + sgn * (ux * ux + uy * uy) * phi)
           + ux * h[1] + uy * h[2];
    h[4] = omega[3] / 4.0 * (-(kxx - kyy) + 2.0 * (ux * kx - uy * ky)
                             + sgn * (ux * ux - uy * uy) * phi)
           + ux * h[1] - uy * h[2];
    /* Eq. (48). */
    orc_d2q5_apply_l(g, h, gp);
}

/* ------------------------------------------------------------------------ */
/* Lattice-independent pseudo-central construction (D2Q9 and D3Q27)           */
/* ------------------------------------------------------------------------ */

typedef struct {
    int q, d;
    int exps[27][3];        /* moment k has exponents exps[k][axis] in {0,1,2} */
    double m[27][27];       /* raw-moment matrix: m[k][alpha] = prod e^exp     */
    double minv[27][27];    /* its inverse                                      */
    double norm_ex;         /* <e_x|e_x>                                        */
    int ready;
} generic_lattice;

static generic_lattice g_lat[3];

static double ipow(double b, int e) {
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

/* Gauss-Jordan inverse with partial pivoting. */
static int invert(int n, double a[27][27], double inv[27][27]) {
    double w[27][54];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j) w[i][j] = (j < n) ? a[i][j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(w[r][c]) > fabs(w[piv][c])) piv = r;
        if (fabs(w[piv][c]) < 1e-12) return -1;
        if (piv != c)
            for (int j = 0; j < 2 * n; ++j) { double t = w[c][j]; w[c][j] = w[piv][j]; w[piv][j] = t; }
        double p = w[c][c];
        for (int j = 0; j < 2 * n; ++j) w[c][j] /= p;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double s = w[r][c];
            if (s == 0.0) continue;
            for (int j = 0; j < 2 * n; ++j) w[r][j] -= s * w[c][j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) inv[i][j] = w[i][j + n];
    return 0;
}

static const generic_lattice* get_generic(int lattice) {
    int key = lattice == ORC_D3Q27 ? 2 : 0;
    generic_lattice* L = &g_lat[key];
    if (L->ready) return L;
    int lat = lattice == ORC_D3Q27 ? ORC_D3Q27 : ORC_D2Q9;
    L->q = orc_num_dirs(lat);
    L->d = orc_num_dims(lat);
    for (int k = 0; k < L->q; ++k) {
        int r = k;
        for (int i = 0; i < 3; ++i) {
            L->exps[k][i] = (i < L->d) ? r % 3 : 0;
            r /= 3;
        }
    }
    for (int k = 0; k < L->q; ++k)
        for (int a = 0; a < L->q; ++a) {
            double v = 1.0;
            for (int i = 0; i < L->d; ++i) v *= ipow((double)orc_velocity(lat, a, i), L->exps[k][i]);
            L->m[k][a] = v;
        }
    invert(L->q, L->m, L->minv);
    L->norm_ex = 0.0;
    for (int a = 0; a < L->q; ++a) L->norm_ex += ipow((double)orc_velocity(lat, a, 0), 2);
    L->ready = 1;
    return L;
}

static double binom2(int n, int k) { return (n == 2 && k == 1) ? 2.0 : 1.0; }

/* Shift raw-type moments by velocity v: out_k = sum_{k' <= k} prod C(a,a') (-v)^(a-a') in_k'. */
static void shift_moments(const generic_lattice* L, const double v[3], const double* in, double* out) {
    for (int k = 0; k < L->q; ++k) {
        double acc = 0.0;
        for (int kp = 0; kp < L->q; ++kp) {
            double c = 1.0;
            for (int i = 0; i < L->d; ++i) {
                int a = L->exps[k][i], ap = L->exps[kp][i];
                if (ap > a) { c = 0.0; break; }
                c *= binom2(a, ap) * ipow(-v[i], a - ap);
            }
            if (c != 0.0) acc += c * in[kp];
        }
        out[k] = acc;
    }
}

/*
 * Generic cascaded collision + Strang forcing for one node.
 *   lattice : ORC_D2Q9 or ORC_D3Q27 (population order as in orc_velocity)
 *   rates   : [omega_bulk, omega_shear, omega_third, omega_fourth_and_higher]
 */
void orc_generic_collide(int lattice, const double* f, const double* fpre, const double* ftot,
                         const double rates[4], double* fp, double* u_out) {
    const generic_lattice* L = get_generic(lattice);
    int q = L->q, d = L->d;
    double m[27], mt[27], kap[27], kpost[27], mpost[27], u[3] = {0, 0, 0};
    for (int k = 0; k < q; ++k) {
        double acc = 0.0;
        for (int a = 0; a < q; ++a) acc += L->m[k][a] * f[a];
        m[k] = acc;
    }
    double rho = m[0];
    /* Pre-collision half force step; the first raw moments become rho*u. */
    memcpy(mt, m, sizeof(double) * q);
    for (int i = 0; i < d; ++i) {
        int k1 = (i == 0) ? 1 : (i == 1 ? 3 : 9);
        u[i] = (m[k1] + 0.5 * fpre[i]) / rho;
        mt[k1] = rho * u[i];
    }
    if (u_out)
        for (int i = 0; i < d; ++i) u_out[i] = u[i];
    shift_moments(L, u, mt, kap);

    double wb = rates[0], ws = rates[1], w3 = rates[2], w4 = rates[3];
    /* Central-moment equilibria (eq. (20) and its 3D analogue). */
    double keq[27];
    for (int k = 0; k < q; ++k) {
        double v = rho;
        for (int i = 0; i < d; ++i) {
            int a = L->exps[k][i];
            v *= (a == 0) ? 1.0 : (a == 2 ? 1.0 / 3.0 : 0.0);
        }
        keq[k] = v;
    }
    for (int k = 0; k < q; ++k) {
        int order = 0, ntwo = 0;
        for (int i = 0; i < d; ++i) { order += L->exps[k][i]; ntwo += (L->exps[k][i] == 2); }
        if (order == 0) kpost[k] = rho;
        else if (order == 1) kpost[k] = 0.0;
        else if (order == 2 && ntwo == 0) kpost[k] = kap[k] + ws * (keq[k] - kap[k]);
        else if (order == 2) kpost[k] = kap[k]; /* diagonal: handled below */
        else if (order == 3) kpost[k] = kap[k] + w3 * (keq[k] - kap[k]);
        else kpost[k] = kap[k] + w4 * (keq[k] - kap[k]);
    }
    /* Diagonal second order: trace relaxed with the bulk rate, deviators with
     * the shear rate. */
    int kd[3];
    kd[0] = 2; kd[1] = 6; kd[2] = 18;
    double tr = 0.0, treq = 0.0;
    for (int i = 0; i < d; ++i) { tr += kap[kd[i]]; treq += keq[kd[i]]; }
    double trp = tr + wb * (treq - tr);
    double devp[3] = {0, 0, 0};
    for (int i = 1; i < d; ++i) devp[i] = (1.0 - ws) * (kap[kd[0]] - kap[kd[i]]);
    double first = trp;
    for (int i = 1; i < d; ++i) first += devp[i];
    first /= (double)d;
    kpost[kd[0]] = first;
    for (int i = 1; i < d; ++i) kpost[kd[i]] = first - devp[i];

    double mu[3] = {-u[0], -u[1], -u[2]};
    shift_moments(L, mu, kpost, mpost);
    double dm[27];
    for (int k = 0; k < q; ++k) dm[k] = mpost[k] - mt[k];
    for (int a = 0; a < q; ++a) {
        double acc = 0.0;
        for (int k = 0; k < q; ++k) acc += L->minv[a][k] * dm[k];
        double kick = 0.0;
        for (int i = 0; i < d; ++i) kick += ftot[i] * (double)orc_velocity(lattice, a, i);
        fp[a] = f[a] + acc + kick / L->norm_ex;
    }
}

/* Raw-moment matrix of the generic construction, for tests. */
void orc_generic_matrix(int lattice, double* m_out, double* minv_out, int* exps_out) {
    const generic_lattice* L = get_generic(lattice);
    for (int k = 0; k < L->q; ++k)
        for (int a = 0; a < L->q; ++a) {
            m_out[k * L->q + a] = L->m[k][a];
            minv_out[k * L->q + a] = L->minv[k][a];
        }
    for (int k = 0; k < L->q; ++k)
        for (int i = 0; i < 3; ++i) exps_out[k * 3 + i] = L->exps[k][i];
}

/* ------------------------------------------------------------------------ */
/* Equilibrium (initial state)                                                */
/* ------------------------------------------------------------------------ */

/* One-dimensional factor of the product-form equilibrium whose central
 * moments are (1, 0, 1/3) along each axis (eq. (20)). */
static double psi(int e, double u) {
    if (e == 0) return 2.0 / 3.0 - u * u;
    return (1.0 / 3.0 + u * u + e * u) / 2.0;
}

void orc_flow_equilibrium(int lattice, double rho, const double* u, double* feq) {
    int q = orc_num_dirs(lattice), d = orc_num_dims(lattice);
    if (lattice == ORC_D3Q15) {
        /* not a tensor-product lattice: the standard second-order equilibrium
         * w_a rho (1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u.u), w = 2/9, 1/9, 1/72 */
        const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        for (int a = 0; a < q; ++a) {
            const int e2 = D3Q15_EX[a] * D3Q15_EX[a] + D3Q15_EY[a] * D3Q15_EY[a] + D3Q15_EZ[a] * D3Q15_EZ[a];
            const double w = e2 == 0 ? 2.0 / 9.0 : (e2 == 1 ? 1.0 / 9.0 : 1.0 / 72.0);
            const double eu = D3Q15_EX[a] * u[0] + D3Q15_EY[a] * u[1] + D3Q15_EZ[a] * u[2];
            feq[a] = w * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
        }
        return;
    }
    for (int a = 0; a < q; ++a) {
        double v = rho;
        for (int i = 0; i < d; ++i) v *= psi(orc_velocity(lattice, a, i), u[i]);
        feq[a] = v;
    }
}

/* D2Q5 equilibrium whose central moments are those of eq. (39). */
void orc_scalar_equilibrium(double phi, const double u[2], double geq[5]) {
    double ux = u[0], uy = u[1];
    geq[0] = phi * (1.0 / 3.0 - ux * ux - uy * uy);
    geq[1] = phi * (1.0 / 3.0 + ux * ux + ux) / 2.0;
    geq[2] = phi * (1.0 / 3.0 + uy * uy + uy) / 2.0;
    geq[3] = phi * (1.0 / 3.0 + ux * ux - ux) / 2.0;
    geq[4] = phi * (1.0 / 3.0 + uy * uy - uy) / 2.0;
}

/* ------------------------------------------------------------------------ */
/* D3Q15 cascaded collision with Strang forcing (Appendix A)                  */
/* ------------------------------------------------------------------------ */

/* Orthogonal basis of eq. (2A): K[beta][alpha]. */
void orc_d3q15_basis(double K[15][15]) {
    for (int a = 0; a < 15; ++a) {
        const double x = D3Q15_EX[a], y = D3Q15_EY[a], z = D3Q15_EZ[a];
        const double e2 = x * x + y * y + z * z;
        K[0][a] = 1.0;
        K[1][a] = x;
        K[2][a] = y;
        K[3][a] = z;
        K[4][a] = x * y;
        K[5][a] = x * z;
        K[6][a] = y * z;
        K[7][a] = x * x - y * y;
        K[8][a] = e2 - 3.0 * z * z;
        K[9][a] = e2 - 2.0;
        K[10][a] = 5.0 * x * e2 - 13.0 * x;
        K[11][a] = 5.0 * y * e2 - 13.0 * y;
        K[12][a] = 5.0 * z * e2 - 13.0 * z;
        K[13][a] = x * y * z;
        K[14][a] = 30.0 * (x * x * y * y + x * x * z * z + y * y * z * z) - 40.0 * e2 + 32.0;
    }
}

/*
 * D3Q15 update of one node (Appendix A): streamed populations f, forces
 * (fpre, ftot); rates w[0] = shear (omega_4..omega_8), w[1] = bulk
 * (omega_9), w[2] = third order (omega_10..omega_13), w[3] = fourth order
 * (omega_14).  Output post-collision populations fp and the half-forced u.
 *  - u from eq. (8A); the collision changes g_4..g_14 of eq. (6A), with
 *    the raw moments (primed kappas) of the streamed populations;
 *  - g_1..g_3 = F_tot/10 (eq. (13A)), g_0 = 0;
 *  - f^p = f + K g, K of eq. (2A).
 * Readings of eq. (6A): g_8 is taken with its closing bracket; g_9 relaxes
 * the trace of the second central moments towards its equilibrium rho
 * (3 c_s^2 rho), so its bracket carries +rho, as g_3 of eq. (23) carries
 * (2/3) rho = 2 c_s^2 rho in 2D (printed without it, the trace would relax
 * to zero); the undefined product term of g_14 is the fourth-order central
 * equilibrium rho c_s^4 = rho/9 (as rho/9 in g_8 of eq. (23)) -- no result
 * printed in the paper pins this term.
 */
void orc_d3q15_collide(const double* f, const double* fpre, const double* ftot, const double w[4], double* fp,
                       double* u_out) {
    double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    double kxy = 0, kxz = 0, kyz = 0, kxx = 0, kyy = 0, kzz = 0, kxyy = 0, kxxy = 0, kxxz = 0, kxyz = 0, kxxyy = 0;
    for (int a = 0; a < 15; ++a) {
        const double x = D3Q15_EX[a], y = D3Q15_EY[a], z = D3Q15_EZ[a], v = f[a];
        rho += v;
        jx += v * x;
        jy += v * y;
        jz += v * z;
        kxy += v * x * y;
        kxz += v * x * z;
        kyz += v * y * z;
        kxx += v * x * x;
        kyy += v * y * y;
        kzz += v * z * z;
        kxyy += v * x * y * y;
        kxxy += v * x * x * y;
        kxxz += v * x * x * z;
        kxyz += v * x * y * z;
        kxxyy += v * x * x * y * y;
    }
    const double ux = (jx + 0.5 * fpre[0]) / rho, uy = (jy + 0.5 * fpre[1]) / rho, uz = (jz + 0.5 * fpre[2]) / rho;
    const double ws = w[0], wb = w[1], w3 = w[2], w4 = w[3];
    double g[15];
    g[0] = 0.0;
    g[1] = ftot[0] / 10.0;
    g[2] = ftot[1] / 10.0;
    g[3] = ftot[2] / 10.0;
    g[4] = ws / 8.0 * (-kxy + rho * ux * uy);
    g[5] = ws / 8.0 * (-kxz + rho * ux * uz);
    g[6] = ws / 8.0 * (-kyz + rho * uy * uz);
    g[7] = ws / 4.0 * (-(kxx - kyy) + rho * (ux * ux - uy * uy));
    g[8] = ws / 12.0 * (-(kxx + kyy - 2.0 * kzz) + rho * (ux * ux + uy * uy - 2.0 * uz * uz));
    g[9] = wb / 18.0 * (rho - (kxx + kyy + kzz) + rho * (ux * ux + uy * uy + uz * uz));
    g[10] = w3 / 16.0 * (-kxyy + 2.0 * uy * kxy + ux * kyy - 2.0 * rho * ux * uy * uy) + uy * g[4] +
            ux * (-g[7] + g[8] + 3.0 * g[9]) / 8.0;
    g[11] = w3 / 16.0 * (-kxxy + 2.0 * ux * kxy + uy * kxx - 2.0 * rho * ux * ux * uy) + ux * g[4] +
            uy * (g[7] + g[8] + 3.0 * g[9]) / 8.0;
    g[12] = w3 / 16.0 * (-kxxz + 2.0 * ux * kxz + uz * kxx - 2.0 * rho * ux * ux * uz) + ux * g[5] +
            uz * (g[7] + g[8] + 3.0 * g[9]) / 8.0;
    g[13] = w3 / 8.0 * (-kxyz + ux * kyz + uy * kxz + uz * kxy - 2.0 * rho * ux * uy * uz) + uz * g[4] +
            uy * g[5] + ux * g[6];
    g[14] = w4 / 16.0 * (-kxxyy + 2.0 * ux * kxyy + 2.0 * uy * kxxy - ux * ux * kyy - uy * uy * kxx -
                         4.0 * ux * uy * kxy + rho / 9.0 + 3.0 * rho * ux * ux * uy * uy) -
            2.0 * ux * uy * g[4] + (ux * ux - uy * uy) * g[7] / 8.0 + (-ux * ux - uy * uy) * g[8] / 8.0 +
            (3.0 / 8.0 * (-ux * ux - uy * uy) - 0.5) * g[9] + 2.0 * ux * g[10] + 2.0 * uy * g[11];
    double K[15][15];
    orc_d3q15_basis(K);
    for (int a = 0; a < 15; ++a) {
        double s = f[a];
        for (int b = 0; b < 15; ++b) s += K[b][a] * g[b];
        fp[a] = s;
    }
    u_out[0] = ux;
    u_out[1] = uy;
    u_out[2] = uz;
}

/* ------------------------------------------------------------------------ */
/* Domain                                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t lattice;
    int32_t d2q9_generic;      /* 1: D2Q9 flow through the generic construction */
    int32_t d2q5_printed_sign; /* 1: eq. (41) with the printed sign            */
    int32_t nthreads;          /* OpenMP threads (0 = runtime default)          */
    int64_t nx, ny, nz;
    int32_t bc_lo[3], bc_hi[3];
    double omega_bulk, omega_shear, omega_third, omega_fourth;
    double omega_phi_diff, omega_phi_high;
    double force[3];
    const double* force_field;  /* [dims][N] or NULL (then `force` is used) */
    int32_t force_time_mode;
    double force_omega;
    double source;
    const double* source_field; /* [N] or NULL */
    int32_t source_time_mode;
    double source_omega;
    double lorentz;             /* sigma B0^2: x-force F_x - lorentz * u_x (Hartmann flow) */
    /* walls (sides with bc = ORC_BOUNCE_BACK), index [axis][0 = low, 1 = high] */
    double wall_u[3][2][3];     /* wall velocity: moving-wall bounce-back of the flow     */
    int32_t phi_wall[3][2];     /* scalar: 0 = bounce-back (no flux), 1 = fixed value      */
    double phi_wall_value[3][2];
    double viscous_heating;     /* c_h: scalar source c_h (S:S) from the flow's strain rate */
} orc_params;

/*
 * Velocity-dependent force F_x(u) = Fb_x - lorentz * u_x (Lorentz force of a
 * transverse field, Sec. 6 Hartmann flow).  The paper states that such a force
 * makes eq. (13) an implicit equation for u; the half steps are taken as the
 * implicit midpoint rule: the pre-collision half step solves
 * rho u_x = j_x + (Fb_pre,x - lorentz u_x)/2, and the whole step changes the
 * momentum by Fb_tot,x - lorentz u_x with that u.  Returns the forces to use
 * as (fpre, ftot) so that (j + fpre/2)/rho is that u.
 */
static void lorentz_forces(const double* f, int lat, double lorentz, const double* fb_pre, const double* fb_tot,
                           int d, double* fpre, double* ftot) {
    int q = orc_num_dirs(lat);
    double rho = 0.0, jx = 0.0;
    for (int a = 0; a < q; ++a) {
        rho += f[a];
        jx += f[a] * orc_velocity(lat, a, 0);
    }
    double ux = (jx + 0.5 * fb_pre[0]) / (rho + 0.5 * lorentz);
    for (int i = 0; i < d; ++i) {
        fpre[i] = fb_pre[i];
        ftot[i] = fb_tot[i];
    }
    fpre[0] = fb_pre[0] - lorentz * ux;
    ftot[0] = fb_tot[0] - lorentz * ux;
}

/* Trapezoidal averages of the time factor over the two half steps of step n
 * (the step covers [n, n+1]). */
void orc_time_factors(int mode, double omega, int64_t n, double* c_pre, double* c_post) {
    if (mode == ORC_TIME_COS) {
        double t0 = (double)n, th = (double)n + 0.5, t1 = (double)n + 1.0;
        *c_pre = 0.5 * (cos(omega * t0) + cos(omega * th));
        *c_post = 0.5 * (cos(omega * th) + cos(omega * t1));
    } else {
        *c_pre = 1.0;
        *c_post = 1.0;
    }
}

/* The flow lattice of a domain (the coupled 2D lattice flows on D2Q9). */
static int flow_lattice(const orc_params* p) { return p->lattice == ORC_D2Q9_D2Q5 ? ORC_D2Q9 : p->lattice; }

static int64_t node_index(const orc_params* p, int64_t x, int64_t y, int64_t z) {
    return x + p->nx * (y + p->ny * z);
}

/* Rest-state weight of flow direction a: prod_i psi(e_ai, 0), psi(0, 0) = 2/3,
 * psi(+-1, 0) = 1/6 (the product-form equilibrium at rest). */
static double rest_weight(int lat, int a) {
    double w = 1.0;
    for (int i = 0; i < orc_num_dims(lat); ++i) w *= orc_velocity(lat, a, i) == 0 ? 2.0 / 3.0 : 1.0 / 6.0;
    return w;
}

/* The wall side a pull from (x, y, z) along velocity e crosses first (axes in
 * the order x, y, z): returns 1 and (axis, side), or 0 if none. */
static int crossed_side(const orc_params* p, const int64_t c[3], const int e[3], int* axis, int* side) {
    const int64_t n[3] = {p->nx, p->ny, p->nz};
    for (int i = 0; i < 3; ++i) {
        int64_t s = c[i] - e[i];
        if (s < 0 && p->bc_lo[i] == ORC_BOUNCE_BACK) { *axis = i; *side = 0; return 1; }
        if (s >= n[i] && p->bc_hi[i] == ORC_BOUNCE_BACK) { *axis = i; *side = 1; return 1; }
    }
    return 0;
}

/* Source coordinate of a pull along one axis; returns 1 when it lies in a wall. */
static int pull_coord(int64_t c, int e, int64_t n, int bc_lo, int bc_hi, int64_t* out) {
    int64_t s = c - e;
    if (s < 0) {
        if (bc_lo == ORC_BOUNCE_BACK) return 1;
        s += n;
    } else if (s >= n) {
        if (bc_hi == ORC_BOUNCE_BACK) return 1;
        s -= n;
    }
    *out = s;
    return 0;
}

/* Eq. (22b) as a pull: f_alpha(x) = f^p_alpha(x - e_alpha); a link whose source
 * lies in a wall returns the opposite post-collision population of the same
 * node (halfway bounce-back), plus 6 w_alpha rho0 (e_alpha . u_w) when that
 * wall moves with velocity u_w (moving-wall bounce-back, rho0 = 1). */
static void gather_flow(const orc_params* p, const double* fp, int64_t x, int64_t y, int64_t z,
                        double* out) {
    int lat = flow_lattice(p);
    int q = orc_num_dirs(lat);
    int64_t n = p->nx * p->ny * p->nz;
    int64_t here = node_index(p, x, y, z);
    for (int a = 0; a < q; ++a) {
        int64_t sx = x, sy = y, sz = z;
        int wall = 0;
        wall |= pull_coord(x, orc_velocity(lat, a, 0), p->nx, p->bc_lo[0], p->bc_hi[0], &sx);
        wall |= pull_coord(y, orc_velocity(lat, a, 1), p->ny, p->bc_lo[1], p->bc_hi[1], &sy);
        wall |= pull_coord(z, orc_velocity(lat, a, 2), p->nz, p->bc_lo[2], p->bc_hi[2], &sz);
        if (wall) {
            out[a] = fp[(int64_t)opposite_dir(lat, a) * n + here];
            const int64_t c[3] = {x, y, z};
            const int e[3] = {orc_velocity(lat, a, 0), orc_velocity(lat, a, 1), orc_velocity(lat, a, 2)};
            int ax = 0, sd = 0;
            if (crossed_side(p, c, e, &ax, &sd)) {
                const double* uw = p->wall_u[ax][sd];
                out[a] += 6.0 * rest_weight(lat, a) * (e[0] * uw[0] + e[1] * uw[1] + e[2] * uw[2]);
            }
        } else {
            out[a] = fp[(int64_t)a * n + node_index(p, sx, sy, sz)];
        }
    }
}

/* Pull of the scalar populations.  A wall link returns the opposite population
 * (bounce-back: no flux) or, on a fixed-value side, minus it plus twice the
 * even part of the equilibrium at the wall value phi_w:
 * g_a = -g^p_opp(a) + phi_w (1/3 + u_w,k^2), k the axis of population a
 * (anti-bounce-back; the paper does not state its wall treatment). */
static void gather_scalar(const orc_params* p, const double* gp, int64_t x, int64_t y, int64_t z,
                          double stot, double* out) {
    int64_t n = p->nx * p->ny * p->nz;
    int64_t here = node_index(p, x, y, z);
    for (int a = 0; a < 5; ++a) {
        int64_t sx = x, sy = y, sz = z;
        int wall = 0;
        wall |= pull_coord(x, D2Q5_EX[a], p->nx, p->bc_lo[0], p->bc_hi[0], &sx);
        wall |= pull_coord(y, D2Q5_EY[a], p->ny, p->bc_lo[1], p->bc_hi[1], &sy);
        if (wall) {
            out[a] = gp[(int64_t)d2q5_opposite(a) * n + here];
            const int64_t c[3] = {x, y, z};
            const int e[3] = {D2Q5_EX[a], D2Q5_EY[a], 0};
            int ax = 0, sd = 0;
            if (crossed_side(p, c, e, &ax, &sd) && p->phi_wall[ax][sd]) {
                const double ua = D2Q5_EX[a] != 0 ? p->wall_u[ax][sd][0] : p->wall_u[ax][sd][1];
                out[a] = -out[a] + p->phi_wall_value[ax][sd] * (1.0 / 3.0 + ua * ua) + 0.4 * stot;
            }
        } else {
            out[a] = gp[(int64_t)a * n + node_index(p, sx, sy, sz)];
        }
    }
}

static void node_force(const orc_params* p, int64_t node, int d, double* f) {
    int64_t n = p->nx * p->ny * p->nz;
    for (int i = 0; i < d; ++i) f[i] = p->force_field ? p->force_field[(int64_t)i * n + node] : p->force[i];
}

static double node_source(const orc_params* p, int64_t node) {
    return p->source_field ? p->source_field[node] : p->source;
}

static void flow_rates_d2q9(const orc_params* p, double w[6]) {
    w[0] = p->omega_bulk;
    w[1] = p->omega_shear;
    w[2] = p->omega_shear;
    w[3] = p->omega_third;
    w[4] = p->omega_third;
    w[5] = p->omega_fourth;
}

/*
 * S:S of the flow's strain-rate tensor S = (grad u + grad u^T)/2 at a node,
 * from the non-equilibrium second moments of the streamed populations f and
 * the half-forced velocity u (Sec. 6, thermal Couette flow): with
 * Pi_ab = sum f e_a e_b - rho u_a u_b - rho/3 delta_ab,
 *   S_xy = -3 w_shear / (2 rho0) Pi_xy                    (as printed),
 *   S_xx - S_yy = -3 w_shear / (2 rho0) (Pi_xx - Pi_yy),
 *   S_xx + S_yy = -3 w_bulk / (2 rho0) (Pi_xx + Pi_yy)
 * (the same first-order relation for each second-order moment with its own
 * relaxation rate), rho0 = 1.  D2Q9 only.
 */
static double strain_rate_squared(const orc_params* p, const double* f, const double* u) {
    double rho = 0.0, kxx = 0.0, kyy = 0.0, kxy = 0.0;
    for (int a = 0; a < 9; ++a) {
        const double ex = orc_velocity(ORC_D2Q9, a, 0), ey = orc_velocity(ORC_D2Q9, a, 1);
        rho += f[a];
        kxx += f[a] * ex * ex;
        kyy += f[a] * ey * ey;
        kxy += f[a] * ex * ey;
    }
    const double pxx = kxx - rho * u[0] * u[0] - rho / 3.0;
    const double pyy = kyy - rho * u[1] * u[1] - rho / 3.0;
    const double pxy = kxy - rho * u[0] * u[1];
    const double sxy = -1.5 * p->omega_shear * pxy;
    const double dif = -1.5 * p->omega_shear * (pxx - pyy);
    const double tr = -1.5 * p->omega_bulk * (pxx + pyy);
    const double sxx = 0.5 * (tr + dif), syy = 0.5 * (tr - dif);
    return sxx * sxx + syy * syy + 2.0 * sxy * sxy;
}

/* Source of the scalar at a node for step n: the prescribed source with its
 * time factors (trapezoid averages of the two half steps), plus the viscous
 * heating c_h (S:S) of the streamed flow populations f and the half-forced
 * velocity u, constant over the step. */
static void scalar_sources(const orc_params* p, int64_t node, const double* f, const double* u, double cs_pre,
                           double cs_post, double* spre, double* stot) {
    const double sb = node_source(p, node);
    *spre = cs_pre * sb;
    *stot = 0.5 * (cs_pre + cs_post) * sb;
    if (p->viscous_heating != 0.0) {
        const double sr = p->viscous_heating * strain_rate_squared(p, f, u);
        *spre += sr;
        *stot += sr;
    }
}

/* One node of one step: pull, then the lattice update; writes the new
 * post-collision populations of this node into f_out / g_out. */
static void step_node(const orc_params* p, const double* f_in, const double* g_in, double* f_out,
                      double* g_out, int64_t x, int64_t y, int64_t z, double cf_pre, double cf_post,
                      double cs_pre, double cs_post) {
    int lat = flow_lattice(p);
    int q = orc_num_dirs(lat), d = orc_num_dims(lat);
    int64_t n = p->nx * p->ny * p->nz;
    int64_t node = node_index(p, x, y, z);
    double f[27], fp[27], fb[3], fpre[3], ftot[3], u[3] = {0, 0, 0};
    gather_flow(p, f_in, x, y, z, f);
    node_force(p, node, d, fb);
    for (int i = 0; i < d; ++i) {
        fpre[i] = cf_pre * fb[i];
        ftot[i] = 0.5 * (cf_pre + cf_post) * fb[i];
    }
    if (p->lorentz != 0.0) {
        double bp[3] = {fpre[0], fpre[1], fpre[2]}, bt[3] = {ftot[0], ftot[1], ftot[2]};
        lorentz_forces(f, lat, p->lorentz, bp, bt, d, fpre, ftot);
    }
    if (lat == ORC_D2Q9 && !p->d2q9_generic) {
        double w[6];
        flow_rates_d2q9(p, w);
        orc_d2q9_collide(f, fpre, ftot, w, fp, u);
    } else if (lat == ORC_D3Q15) {
        double rates[4] = {p->omega_shear, p->omega_bulk, p->omega_third, p->omega_fourth};
        orc_d3q15_collide(f, fpre, ftot, rates, fp, u);
    } else {
        double rates[4] = {p->omega_bulk, p->omega_shear, p->omega_third, p->omega_fourth};
        orc_generic_collide(lat, f, fpre, ftot, rates, fp, u);
    }
    for (int a = 0; a < q; ++a) f_out[(int64_t)a * n + node] = fp[a];
    if (p->lattice == ORC_D2Q9_D2Q5) {
        double g[5], gpo[5], spre, stot;
        scalar_sources(p, node, f, u, cs_pre, cs_post, &spre, &stot);
        gather_scalar(p, g_in, x, y, z, stot, g);
        double w[4] = {p->omega_phi_diff, p->omega_phi_diff, p->omega_phi_high, p->omega_phi_high};
        orc_d2q5_collide(g, u, spre, stot, w, p->d2q5_printed_sign, gpo);
        for (int a = 0; a < 5; ++a) g_out[(int64_t)a * n + node] = gpo[a];
    }
}

#ifdef _OPENMP
#include <omp.h>
#endif

/*
 * Advance the stored post-collision state (f, g) from step n0 by nsteps steps,
 * in place.  f is [Q][N], g is [5][N] (or NULL), N = nx*ny*nz, x fastest.
 */
int orc_run(const orc_params* p, double* f, double* g, int64_t n0, int64_t nsteps) {
    int lat = flow_lattice(p);
    int q = orc_num_dirs(lat);
    int64_t n = p->nx * p->ny * p->nz;
    double* f2 = (double*)malloc(sizeof(double) * (size_t)(q * n));
    double* g2 = NULL;
    if (!f2) return -1;
    if (p->lattice == ORC_D2Q9_D2Q5) {
        g2 = (double*)malloc(sizeof(double) * (size_t)(5 * n));
        if (!g2) { free(f2); return -1; }
    }
    get_generic(lat);
#ifdef _OPENMP
    int nthr = p->nthreads > 0 ? p->nthreads : omp_get_max_threads();
#endif
    double* fa = f;
    double* fb = f2;
    double* ga = g;
    double* gb = g2;
    for (int64_t s = 0; s < nsteps; ++s) {
        double cfp, cfq, csp, csq;
        orc_time_factors(p->force_time_mode, p->force_omega, n0 + s, &cfp, &cfq);
        orc_time_factors(p->source_time_mode, p->source_omega, n0 + s, &csp, &csq);
        int64_t rows = p->ny * p->nz;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthr)
#endif
        for (int64_t r = 0; r < rows; ++r) {
            int64_t y = r % p->ny, z = r / p->ny;
            for (int64_t x = 0; x < p->nx; ++x) step_node(p, fa, ga, fb, gb, x, y, z, cfp, cfq, csp, csq);
        }
        double* t = fa; fa = fb; fb = t;
        t = ga; ga = gb; gb = t;
    }
    if (fa != f) memcpy(f, fa, sizeof(double) * (size_t)(q * n));
    if (g && ga != g) memcpy(g, ga, sizeof(double) * (size_t)(5 * n));
    free(f2);
    free(g2);
    return 0;
}

/*
 * Macroscopic readout of the stored state at step counter n: pull, then
 * rho, the output velocity of eq. (24) (kind 0) or the half-forced velocity of
 * eq. (25) (kind 1), and the scalar of eq. (42) (kind 0) or eq. (43) (kind 1).
 * rho is [N], u is [dims][N], phi is [N] (may be NULL).
 */
int orc_moments(const orc_params* p, const double* f, const double* g, int64_t n, int kind,
                double* rho_out, double* u_out, double* phi_out) {
    int lat = flow_lattice(p);
    int q = orc_num_dirs(lat), d = orc_num_dims(lat);
    int64_t nn = p->nx * p->ny * p->nz;
    double cfp, cfq, csp, csq;
    orc_time_factors(p->force_time_mode, p->force_omega, n, &cfp, &cfq);
    orc_time_factors(p->source_time_mode, p->source_omega, n, &csp, &csq);
    for (int64_t z = 0; z < p->nz; ++z)
        for (int64_t y = 0; y < p->ny; ++y)
            for (int64_t x = 0; x < p->nx; ++x) {
                int64_t node = node_index(p, x, y, z);
                double fl[27], fb[3];
                gather_flow(p, f, x, y, z, fl);
                node_force(p, node, d, fb);
                double rho = 0.0, uh[3] = {0.0, 0.0, 0.0};
                for (int a = 0; a < q; ++a) rho += fl[a];
                rho_out[node] = rho;
                for (int i = 0; i < d; ++i) {
                    double j = 0.0;
                    for (int a = 0; a < q; ++a) j += fl[a] * orc_velocity(lat, a, i);
                    /* half-forced velocity (eq. 25; implicit half step for the Lorentz force) */
                    uh[i] = (j + 0.5 * cfp * fb[i]) / (rho + (i == 0 ? 0.5 * p->lorentz : 0.0));
                    u_out[(int64_t)i * nn + node] = kind == 1 ? uh[i] : j / rho;
                }
                if (p->lattice == ORC_D2Q9_D2Q5 && phi_out && g) {
                    double gl[5], phi = 0.0, spre, stot;
                    scalar_sources(p, node, fl, uh, csp, csq, &spre, &stot);
                    gather_scalar(p, g, x, y, z, stot, gl);
                    for (int a = 0; a < 5; ++a) phi += gl[a];
                    if (kind == 1) phi += 0.5 * spre;
                    phi_out[node] = phi;
                }
            }
    return 0;
}

/*
 * S:S of the flow's strain-rate tensor at every node of the stored state at
 * step counter n, i.e. the viscous-heating source per unit coefficient c_h
 * (Sec. 6, thermal Couette flow): pull, half-forced velocity of eq. (25), then
 * strain_rate_squared on the streamed populations.  D2Q9 flow only (the
 * D2Q9 and D2Q9+D2Q5 lattices); out is [N].  Returns -1 on another lattice.
 */
int orc_strain_rate_field(const orc_params* p, const double* f, int64_t n, double* out) {
    if (flow_lattice(p) != ORC_D2Q9) return -1;
    double cfp, cfq;
    orc_time_factors(p->force_time_mode, p->force_omega, n, &cfp, &cfq);
    for (int64_t z = 0; z < p->nz; ++z)
        for (int64_t y = 0; y < p->ny; ++y)
            for (int64_t x = 0; x < p->nx; ++x) {
                const int64_t node = node_index(p, x, y, z);
                double fl[27], fb[3], uh[3] = {0.0, 0.0, 0.0};
                gather_flow(p, f, x, y, z, fl);
                node_force(p, node, 2, fb);
                double rho = 0.0;
                for (int a = 0; a < 9; ++a) rho += fl[a];
                for (int i = 0; i < 2; ++i) {
                    double j = 0.0;
                    for (int a = 0; a < 9; ++a) j += fl[a] * orc_velocity(ORC_D2Q9, a, i);
                    uh[i] = (j + 0.5 * cfp * fb[i]) / (rho + (i == 0 ? 0.5 * p->lorentz : 0.0));
                }
                out[node] = strain_rate_squared(p, fl, uh);
            }
    return 0;
}

/* Number of OpenMP threads orc_run uses by default. */
int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
