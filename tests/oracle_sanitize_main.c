/*
 * Host-only driver that exercises every entry point of the FP64 oracle, built
 * together with it (one translation unit) under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py.  Small lattices
 * of every kind, walls on every side, moving walls, fixed scalar walls,
 * viscous heating, force and source fields, oscillating forcing and the
 * Lorentz force; exits non-zero if a result is not finite.
 */
#include "../oracle/casclb_oracle.c"

#include <stdio.h>

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;

static double uniform(void) {
    /* splitmix64 */
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static int all_finite(const double* a, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static int run_case(int lattice, int64_t nx, int64_t ny, int64_t nz, int walls, int extras) {
    orc_params p;
    memset(&p, 0, sizeof(p));
    p.lattice = lattice;
    p.nthreads = 2;
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    for (int i = 0; i < 3; ++i) {
        const int wall = (walls >> i) & 1;
        p.bc_lo[i] = p.bc_hi[i] = wall ? ORC_BOUNCE_BACK : ORC_PERIODIC;
    }
    p.omega_bulk = 1.1;
    p.omega_shear = 1.4;
    p.omega_third = 0.9;
    p.omega_fourth = 1.2;
    p.omega_phi_diff = 1.3;
    p.omega_phi_high = 1.0;
    p.force[0] = 1e-5;
    p.force[1] = -2e-5;
    p.force[2] = 3e-6;
    const int flow = lattice == ORC_D2Q9_D2Q5 ? ORC_D2Q9 : lattice;
    const int q = orc_num_dirs(flow), d = orc_num_dims(flow);
    const int64_t n = nx * ny * nz;
    double* f = malloc(sizeof(double) * (size_t)(q * n));
    double* g = lattice == ORC_D2Q9_D2Q5 ? malloc(sizeof(double) * (size_t)(5 * n)) : NULL;
    double* ff = malloc(sizeof(double) * (size_t)(d * n));
    double* sf = malloc(sizeof(double) * (size_t)n);
    double* rho = malloc(sizeof(double) * (size_t)n);
    double* u = malloc(sizeof(double) * (size_t)(d * n));
    double* phi = malloc(sizeof(double) * (size_t)n);
    double* ss = malloc(sizeof(double) * (size_t)n);
    if (!f || !ff || !sf || !rho || !u || !phi || !ss || (lattice == ORC_D2Q9_D2Q5 && !g)) return 2;
    for (int64_t i = 0; i < d * n; ++i) ff[i] = 1e-5 * (uniform() - 0.5);
    for (int64_t i = 0; i < n; ++i) sf[i] = 1e-4 * (uniform() - 0.5);
    for (int64_t node = 0; node < n; ++node) {
        double uu[3] = {0.02 * (uniform() - 0.5), 0.02 * (uniform() - 0.5), d == 3 ? 0.02 * (uniform() - 0.5) : 0.0};
        double feq[27], geq[5];
        orc_flow_equilibrium(flow, 1.0 + 0.01 * (uniform() - 0.5), uu, feq);
        for (int a = 0; a < q; ++a) f[(int64_t)a * n + node] = feq[a] + 1e-4 * (uniform() - 0.5);
        if (g) {
            orc_scalar_equilibrium(uniform(), uu, geq);
            for (int a = 0; a < 5; ++a) g[(int64_t)a * n + node] = geq[a];
        }
    }
    if (extras) {
        p.force_field = ff;
        p.force_time_mode = ORC_TIME_COS;
        p.force_omega = 0.01;
        if (g) {
            p.source_field = sf;
            p.source_time_mode = ORC_TIME_COS;
            p.source_omega = 0.02;
            p.viscous_heating = 2.0;
        }
        if (d == 2) {
            for (int ax = 0; ax < 2; ++ax)
                for (int sd = 0; sd < 2; ++sd) {
                    if (p.bc_lo[ax] != ORC_BOUNCE_BACK) continue;
                    p.wall_u[ax][sd][1 - ax] = 0.01 * (sd ? -1.0 : 1.0);
                    p.phi_wall[ax][sd] = sd;
                    p.phi_wall_value[ax][sd] = 0.5;
                }
            if (lattice == ORC_D2Q9) p.lorentz = 1e-3;
        }
    } else {
        p.source = 1e-5;
    }
    int rc = orc_run(&p, f, g, 0, 7);
    rc |= orc_moments(&p, f, g, 7, 0, rho, u, g ? phi : NULL);
    rc |= orc_moments(&p, f, g, 7, 1, rho, u, g ? phi : NULL);
    if (flow == ORC_D2Q9) rc |= orc_strain_rate_field(&p, f, 7, ss);
    int ok = rc == 0 && all_finite(f, q * n) && all_finite(rho, n) && all_finite(u, d * n);
    if (g) ok = ok && all_finite(g, 5 * n) && all_finite(phi, n);
    if (flow == ORC_D2Q9) ok = ok && all_finite(ss, n);
    printf("lattice %d %lldx%lldx%lld walls %d extras %d: %s\n", lattice, (long long)nx, (long long)ny,
           (long long)nz, walls, extras, ok ? "ok" : "FAILED");
    free(f);
    free(g);
    free(ff);
    free(sf);
    free(rho);
    free(u);
    free(phi);
    free(ss);
    return ok ? 0 : 1;
}

int main(void) {
    int bad = 0;
    for (int extras = 0; extras < 2; ++extras) {
        bad |= run_case(ORC_D2Q9, 7, 5, 1, 0, extras);
        bad |= run_case(ORC_D2Q9, 6, 9, 1, 3, extras);
        bad |= run_case(ORC_D2Q9_D2Q5, 5, 8, 1, 2, extras);
        bad |= run_case(ORC_D2Q9_D2Q5, 4, 6, 1, 3, extras);
        bad |= run_case(ORC_D3Q27, 5, 4, 3, 6, extras);
        bad |= run_case(ORC_D3Q27, 3, 3, 3, 7, extras);
        bad |= run_case(ORC_D3Q15, 4, 5, 3, 6, extras);
        bad |= run_case(ORC_D3Q15, 3, 4, 5, 1, extras);
    }
    /* per-node entry points and the basis / matrix builders */
    double K[15][15], m[27 * 27], mi[27 * 27];
    int ex[27 * 3];
    orc_d3q15_basis(K);
    orc_generic_matrix(ORC_D3Q27, m, mi, ex);
    orc_generic_matrix(ORC_D2Q9, m, mi, ex);
    double fq[9], gk[9] = {0, 1e-3, -2e-3, 1e-4, 0, 0, 1e-5, -1e-5, 1e-6}, fp[9], u2[2], g5[5], gp[5];
    const double z2[2] = {0, 0}, w6[6] = {1, 1.2, 1.2, 1, 1, 1}, w4[4] = {1.3, 1.3, 1, 1};
    orc_flow_equilibrium(ORC_D2Q9, 1.0, z2, fq);
    orc_d2q9_apply_k(fq, gk, fp);
    orc_d2q9_collide(fq, z2, z2, w6, fp, u2);
    orc_scalar_equilibrium(0.3, z2, g5);
    orc_d2q5_collide(g5, z2, 1e-4, 1e-4, w4, 1, gp);
    orc_d2q5_apply_l(g5, gk, gp);
    bad |= !all_finite(fp, 9) || !all_finite(gp, 5);
    printf("%s\n", bad ? "FAILED" : "all ok");
    return bad;
}
