/* Sanitizer run of the FP64 oracle (test infrastructure): compiled together
 * with the oracle's source under AddressSanitizer and UndefinedBehavior-
 * Sanitizer, it drives every entry point on small grids of each boundary
 * kind, collision, energy form and viscosity law.  Exit status 0 when the
 * run is clean; the sanitizers abort otherwise. */
#include "../../oracle/lbddf_oracle.c"

#include <stdio.h>

static orc_params base(int nx, int ny) {
    orc_params p;
    memset(&p, 0, sizeof(p));
    p.nx = nx;
    p.ny = ny;
    p.energy = ORC_TOTAL;
    p.heating = 1;
    p.correction = 1;
    p.coupled = 1;
    p.collision = ORC_MRT;
    p.visc = ORC_CONST_TAU;
    p.rho_extrap = ORC_RHO_PRESSURE;
    p.rho0 = 1.0;
    p.T0 = 1.0;
    p.R = 1.0 / 3.0;
    p.b = 3.0;
    p.Pr = 0.71;
    p.tau_f = 0.8;
    p.s_q = 1.5;
    p.tau_rho = 1.0;
    p.tau_j = 1.0;
    p.mu_ref = 0.05;
    p.T_ref = 1.0;
    p.visc_n = 1.0;
    p.suth_S = 110.5 / 600.0;
    for (int s = 0; s < 4; ++s) {
        p.side_T[s] = 1.0;
        p.side_period[s] = 1.0;
    }
    return p;
}

static int exercise(const char *name, orc_params p, int steps) {
    orc_grid *g = orc_create(&p);
    if (!g) {
        fprintf(stderr, "%s: orc_create failed\n", name);
        return 1;
    }
    const size_t n = (size_t)p.nx * p.ny;
    double *f[4], *pops = malloc(18 * n * sizeof(double)), out[5];
    for (int k = 0; k < 4; ++k) f[k] = malloc(n * sizeof(double));
    for (size_t i = 0; i < n; ++i) {
        const double s = 1e-3 * sin(0.7 * (double)i);
        f[0][i] = 1.0 + s;
        f[1][i] = 0.5 * s;
        f[2][i] = -0.3 * s;
        f[3][i] = 1.0 + 2.0 * s;
    }
    orc_init(g, f[0], f[1], f[2], f[3]);
    (void)orc_residual(g, 1);
    orc_step(g, steps);
    orc_macros(g, f[0], f[1], f[2], f[3]);
    orc_pops(g, pops);
    orc_set_pops(g, pops);
    orc_diag(g, out);
    const double r = orc_residual(g, 1);
    orc_stream_only(g, 3);
    orc_step(g, 2);
    orc_init(g, NULL, NULL, NULL, NULL);
    orc_step(g, 1);
    double fe[9], he[9], me[9], cv[9], fv[9], fh[9], pc[18], m4[4], tr[12];
    orc_node_feq(g, 1.01, 0.02, -0.01, 1.1, fe);
    orc_node_heq(g, 1.01, 0.02, -0.01, 1.1, he);
    orc_node_meq(g, 1.01, 0.02, -0.01, 1.1, me);
    orc_node_correction(1e-4, -2e-4, cv);
    orc_node_forcing(g, 0.02, -0.01, 0.0, -1e-4, fv, fh);
    for (int a = 0; a < 9; ++a) {
        pc[a] = fe[a];
        pc[9 + a] = he[a];
    }
    orc_node_moments(g, pc, m4);
    orc_node_collide(g, pc, 1e-4, -1e-4, pc);
    orc_node_transport(g, 1.01, 1.1, tr);
    printf("%s: %ld steps, mass %.12f, bad %g, residual %.3e\n", name, orc_time(g), out[0], out[4], r);
    orc_destroy(g);
    for (int k = 0; k < 4; ++k) free(f[k]);
    free(pops);
    return out[4] != 0.0;
}

int main(void) {
    int fails = 0;
    orc_set_threads(1);
    (void)orc_threads();
    {
        orc_params p = base(17, 9);
        fails += exercise("periodic total+heating, MRT", p, 20);
        p.collision = ORC_BGK;
        p.coupled = 0;
        fails += exercise("periodic decoupled, BGK", p, 20);
        fails += exercise("periodic 1x1", base(1, 1), 10);
    }
    {
        orc_params p = base(12, 12);
        p.energy = ORC_INTERNAL;
        p.heating = 0;
        p.visc = ORC_SUTHERLAND;
        p.g = 1e-4;
        p.side_kind[0] = p.side_kind[1] = ORC_WALL;
        p.side_kind[2] = p.side_kind[3] = ORC_ADIABATIC;
        p.side_T[0] = 1.3;
        p.side_T[1] = 0.7;
        fails += exercise("cavity internal, Sutherland, gravity", p, 20);
        p.rho_extrap = ORC_RHO_DENSITY;
        fails += exercise("cavity, density extrapolation", p, 20);
    }
    {
        orc_params p = base(20, 4);
        p.side_kind[0] = ORC_INLET;
        p.side_kind[1] = ORC_OUTLET;
        p.side_amp[0] = 0.01;
        p.side_period[0] = 7.0;
        fails += exercise("channel inlet/outlet", p, 20);
    }
    {
        orc_params p = base(3, 8);
        p.correction = 0;
        p.visc = ORC_POWER;
        p.mu_ref = 0.25;
        p.s_e = p.s_zeta = 1.5;
        p.side_kind[2] = ORC_ADIABATIC;
        p.side_kind[3] = ORC_WALL;
        p.side_ux[3] = 0.1;
        fails += exercise("Couette power law, adiabatic wall", p, 20);
    }
    return fails != 0;
}
