/*
 * FP64 CPU oracle of the coupled double-distribution-function (DDF) thermal
 * lattice Boltzmann model on D2Q9 of Li, Luo, He, Gao & Tao, "Coupling lattice
 * Boltzmann model for simulation of thermal flows on standard lattices".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark load this library.  The product (the HIP library)
 * never calls it and shares no code, header, table or helper with it.
 *
 * Written for readability, not speed:
 *   - array-of-structures state, node-major: pop[(j*nx + i)*18 + k],
 *     k = 0..8 the density populations f^, k = 9..17 the energy populations h-;
 *   - push streaming, one whole-grid pass per stage of a time step;
 *   - the moment transform uses the two matrices of Appendix B as printed
 *     (Eq. B1, B2) through plain 9x9 matrix-vector products;
 *   - everything in double precision, lattice units (dx = dt = c = 1, so that
 *     R T0 = 1/3, Sec. II and Sec. IV-A).
 *
 * One time step n -> n+1 (Sec. III-C-2 with the boundary rules of Sec. IV):
 *   1. moments of every node from its pre-collision populations
 *      (Eq. 46, P-forcing note after Eq. 51, Eq. 37 or the internal-energy
 *      form of Sec. III-C-1);
 *   2. boundary nodes: macroscopic values from the boundary condition and
 *      populations rebuilt by non-equilibrium extrapolation;
 *   3. Q = rho u (1 - theta) everywhere (Eq. 48);
 *   4. collision of every node: correction term (Eq. 48-50), forcing
 *      (Eq. 51), MRT collision of f (Eq. 44) or BGK (Eq. 34), BGK collision
 *      of h with the coupling term (Eq. 47);
 *   5. streaming (Eq. 45) with periodic wrap; populations leaving through a
 *      non-periodic side are dropped.
 *
 * Readings where the paper is silent or garbled (both this oracle and the GPU
 * path follow them):
 *   - Eq. 51: the p_xx entry of F^ is 2(u_x a_x - u_y a_y) (the printed
 *     "u_x a_y" does not follow from M F with the stated F_alpha);
 *   - the walls use non-equilibrium extrapolation from the nearest interior
 *     node along the inward normal (the diagonal neighbour at corners):
 *     pop_b = eq(rho_b,u_b,T_b) + [pop_f - eq(rho_f,u_f,T_f)] for f^ and h-;
 *   - a Dirichlet-temperature wall takes its density from pressure
 *     extrapolation that respects the hydrostatic balance of the body force,
 *     p_b = p_f exp(g (y_f - y_b) / (R (T_f + T_b)/2)) with p = rho R T (so
 *     rho_b = rho_f T_f / T_b without gravity), unless density extrapolation
 *     is asked for (rho_b = rho_f); plain p_b = p_f lets a closed box at rest
 *     under gravity leak mass through its horizontal walls every step;
 *   - an adiabatic wall takes the second-order one-sided zero-gradient value
 *     T_b = (4 T_1 - T_2)/3 from the first two nodes along the inward normal
 *     (the diagonal at corners), and rho_b as for a Dirichlet wall;
 *   - corners take the velocity of the x-side wall and the temperature of a
 *     Dirichlet x-side wall, else of a Dirichlet y-side wall, else T_f;
 *   - the correction term is zero on boundary nodes; their neighbours use
 *     Q_b computed from the boundary values;
 *   - inlet (x = 0): post-collision populations are the equilibria at
 *     u = U0 s, rho = rho0 (1 + U0 s / c_s), T = T0 (1 + (gamma-1) U0 s / c_s),
 *     s = sin(2 pi n / P), c_s = sqrt(gamma R T0) (Eq. 53, 54);
 *   - outlet (x = nx-1): zero gradient, i.e. the node takes the moments and
 *     an exact copy of the populations of node nx-2, then collides;
 *   - Z_alpha = e_alpha . u (the Navier-Stokes-level form, Sec. II);
 *   - tau_h = (tau_f - 1/2)/Pr, omega_h = 2/(2 tau_h + 1),
 *     1/tau_hf = (Pr - 1)/tau_f (Sec. III-C-2);
 *   - the BGK variant uses omega_f = 1/tau_f, i.e. the same viscosity
 *     (tau_f - 1/2) p as the MRT scheme, and the source sign +(1-omega_f/2)C
 *     that follows from Eq. 32-33 (Eq. 34 prints a minus);
 *   - initial populations are the equilibria of the initial fields.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NQ 9
#define DIM 2
#define NPOP 18
/* Grids smaller than this run their passes on one thread: a thread team's
 * start-up and barriers would cost more than the work of a small grid. */
#define ORC_OMP_MIN_NODES 8192

enum { ORC_PERIODIC = 0, ORC_WALL = 1, ORC_ADIABATIC = 2, ORC_INLET = 3, ORC_OUTLET = 4 };
enum { ORC_TOTAL = 0, ORC_INTERNAL = 1 };
enum { ORC_CONST_TAU = 0, ORC_CONST_MU = 1, ORC_POWER = 2, ORC_SUTHERLAND = 3 };
enum { ORC_MRT = 0, ORC_BGK = 1 };
enum { ORC_RHO_PRESSURE = 0, ORC_RHO_DENSITY = 1 };

typedef struct {
    int32_t nx, ny;
    int32_t energy, heating, correction, coupled, collision, visc, rho_extrap, pad_;
    int32_t side_kind[4]; /* x-, x+, y-, y+ */
    double rho0, T0, R, b, Pr, tau_f, s_e, s_zeta, s_q, tau_rho, tau_j;
    double mu_ref, T_ref, visc_n, suth_S, g;
    double side_ux[4], side_uy[4], side_T[4], side_amp[4], side_period[4];
} orc_params;

typedef struct {
    orc_params p;
    int nx, ny;
    long n; /* time step counter */
    double *pop;   /* pre-collision state at time n, [node][18] */
    double *post;  /* scratch: post-collision / streaming target */
    double *rho, *ux, *uy, *T; /* moments after the boundary treatment */
    double *Qx, *Qy;
    double *Tsnap;
    int have_snap;
    int ex[NQ], ey[NQ];
    double w[NQ];
} orc_grid;

/* ---- Appendix B, Eq. B1 and B2, as printed ---------------------------- */
static const double MB1[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
};

static const double MB2[9][9] = {
    {1. / 9, -1. / 9, 1. / 9, 0, 0, 0, 0, 0, 0},
    {1. / 9, -1. / 36, -1. / 18, 1. / 6, -1. / 6, 0, 0, 1. / 4, 0},
    {1. / 9, -1. / 36, -1. / 18, 0, 0, 1. / 6, -1. / 6, -1. / 4, 0},
    {1. / 9, -1. / 36, -1. / 18, -1. / 6, 1. / 6, 0, 0, 1. / 4, 0},
    {1. / 9, -1. / 36, -1. / 18, 0, 0, -1. / 6, 1. / 6, -1. / 4, 0},
    {1. / 9, 1. / 18, 1. / 36, 1. / 6, 1. / 12, 1. / 6, 1. / 12, 0, 1. / 4},
    {1. / 9, 1. / 18, 1. / 36, -1. / 6, -1. / 12, 1. / 6, 1. / 12, 0, -1. / 4},
    {1. / 9, 1. / 18, 1. / 36, -1. / 6, -1. / 12, -1. / 6, -1. / 12, 0, 1. / 4},
    {1. / 9, 1. / 18, 1. / 36, 1. / 6, 1. / 12, -1. / 6, -1. / 12, 0, -1. / 4},
};

static void matvec9(const double A[9][9], const double x[9], double y[9]) {
    for (int r = 0; r < 9; ++r) {
        double s = 0.0;
        for (int c = 0; c < 9; ++c) s += A[r][c] * x[c];
        y[r] = s;
    }
}

/* ---- D2Q9 lattice, Eq. 6 with c = 1, weights as given after Eq. 8 ------- */
static void lattice(int ex[NQ], int ey[NQ], double w[NQ]) {
    ex[0] = 0;
    ey[0] = 0;
    for (int a = 1; a <= 4; ++a) {
        double ang = (a - 1) * M_PI / 2.0;
        ex[a] = (int)lround(cos(ang));
        ey[a] = (int)lround(sin(ang));
    }
    for (int a = 5; a <= 8; ++a) {
        double ang = (2 * a - 1) * M_PI / 4.0;
        ex[a] = (int)lround(sqrt(2.0) * cos(ang));
        ey[a] = (int)lround(sqrt(2.0) * sin(ang));
    }
    w[0] = 4.0 / 9.0;
    for (int a = 1; a <= 4; ++a) w[a] = 1.0 / 9.0;
    for (int a = 5; a <= 8; ++a) w[a] = 1.0 / 36.0;
}

/* ---- equilibria ---------------------------------------------------------- */
/* theta and p entering the equilibria: the coupled model uses theta = T/T0 and
 * p = rho R T (Eq. 18); the decoupled model theta = 1, p = p0 = rho R T0 (Eq. 8). */
static double theta_eq(const orc_grid *g, double T) { return g->p.coupled ? T / g->p.T0 : 1.0; }
static double p_eq(const orc_grid *g, double rho, double T) {
    return g->p.coupled ? rho * g->p.R * T : rho * g->p.R * g->p.T0;
}

/* Eq. 18a */
static void feq(const orc_grid *g, double rho, double ux, double uy, double T, double out[NQ]) {
    const double RT0 = g->p.R * g->p.T0;
    const double th = theta_eq(g, T);
    const double u2 = ux * ux + uy * uy;
    for (int a = 0; a < NQ; ++a) {
        const double eu = g->ex[a] * ux + g->ey[a] * uy;
        const double e2 = (double)(g->ex[a] * g->ex[a] + g->ey[a] * g->ey[a]);
        const double x = eu / RT0;
        out[a] = rho * g->w[a] *
                 (1.0 + x + 0.5 * (x * x - u2 / RT0 + (th - 1.0) * (e2 / RT0 - DIM)) +
                  eu / (2.0 * RT0) * (th - 1.0) * (e2 / RT0 - DIM - 2.0));
    }
}

/* Eq. 18b (total energy E = (b R T + u^2)/2), or the internal-energy form
 * h_eq = b R T f_eq / 2 of Sec. III-C-1. */
static void heq(const orc_grid *g, double rho, double ux, double uy, double T, const double f_eq[NQ],
                double out[NQ]) {
    const double RT0 = g->p.R * g->p.T0;
    if (g->p.energy == ORC_INTERNAL) {
        for (int a = 0; a < NQ; ++a) out[a] = 0.5 * g->p.b * g->p.R * T * f_eq[a];
        return;
    }
    const double th = theta_eq(g, T);
    const double p = p_eq(g, rho, T);
    const double u2 = ux * ux + uy * uy;
    const double E = 0.5 * (g->p.b * g->p.R * T + u2);
    for (int a = 0; a < NQ; ++a) {
        const double eu = g->ex[a] * ux + g->ey[a] * uy;
        const double e2 = (double)(g->ex[a] * g->ex[a] + g->ey[a] * g->ey[a]);
        out[a] = E * f_eq[a] +
                 g->w[a] * p * (eu / RT0 + (eu / RT0) * (eu / RT0) - u2 / RT0 + 0.5 * th * (e2 / RT0 - DIM));
    }
}

/* Eq. 41 (moment-space equilibria, lattice units) */
static void meq(const orc_grid *g, double rho, double ux, double uy, double T, double m[NQ]) {
    const double th = theta_eq(g, T);
    const double u2 = ux * ux + uy * uy;
    m[0] = rho;
    m[1] = rho * (-4.0 + 3.0 * u2 + 2.0 * th);
    m[2] = rho * (3.0 - 3.0 * u2 - 2.0 * th);
    m[3] = rho * ux;
    m[4] = rho * (-2.0 * ux + ux * th);
    m[5] = rho * uy;
    m[6] = rho * (-2.0 * uy + uy * th);
    m[7] = rho * (ux * ux - uy * uy);
    m[8] = rho * ux * uy;
}

/* Eq. 49: velocity-space correction term from phi_x, phi_y */
static void correction_vel(double phix, double phiy, double C[NQ]) {
    C[0] = -phix / 9.0;
    C[1] = -phix / 36.0 + phiy / 4.0;
    C[2] = -phix / 36.0 - phiy / 4.0;
    C[3] = C[1];
    C[4] = C[2];
    C[5] = C[6] = C[7] = C[8] = phix / 18.0;
}

/* Forcing term of Sec. III-C-3: F_a = w_a [e.a / RT0 + u a : (e e - RT0 I) / RT0^2] */
static void forcing_vel(const orc_grid *g, double ux, double uy, double ax, double ay, double F[NQ]) {
    const double RT0 = g->p.R * g->p.T0;
    for (int a = 0; a < NQ; ++a) {
        const double ex = g->ex[a], ey = g->ey[a];
        const double ea = ex * ax + ey * ay;
        /* u a : (e e - RT0 I) = sum_ij u_i a_j (e_i e_j - RT0 delta_ij) */
        const double uaee = (ux * ex + uy * ey) * (ax * ex + ay * ey) - RT0 * (ux * ax + uy * ay);
        F[a] = g->w[a] * (ea / RT0 + uaee / (RT0 * RT0));
    }
}

/* Eq. 51 (moment-space forcing), p_xx entry read as 2(u_x a_x - u_y a_y) */
static void forcing_mom(double ux, double uy, double ax, double ay, double Fh[NQ]) {
    const double ua = ux * ax + uy * ay;
    Fh[0] = 0.0;
    Fh[1] = 6.0 * ua;
    Fh[2] = -6.0 * ua;
    Fh[3] = ax;
    Fh[4] = -ax;
    Fh[5] = ay;
    Fh[6] = -ay;
    Fh[7] = 2.0 * (ux * ax - uy * ay);
    Fh[8] = ux * ay + uy * ax;
}

/* ---- transport (Sec. III-C-2, Sec. IV-A, Eq. 59) ------------------------ */
typedef struct {
    double tau_f, s[NQ], omega_h, inv_tau_hf;
} transport;

static double viscosity(const orc_grid *g, double T) {
    const orc_params *p = &g->p;
    switch (p->visc) {
    case ORC_POWER: return p->mu_ref * pow(T / p->T_ref, p->visc_n);
    case ORC_SUTHERLAND: {
        /* mu/mu* = (T/T*)^{3/2} (T* + S)/(T + S) with mu* fixed by mu(T_ref) = mu_ref;
         * T* cancels out of mu(T)/mu(T_ref). */
        const double r = T / p->T_ref;
        return p->mu_ref * r * sqrt(r) * (p->T_ref + p->suth_S) / (T + p->suth_S);
    }
    default: return p->mu_ref;
    }
}

static void transport_at(const orc_grid *g, double rho, double T, transport *t) {
    const orc_params *p = &g->p;
    if (p->visc == ORC_CONST_TAU) {
        t->tau_f = p->tau_f;
    } else {
        /* tau_f = mu / p + dt/2 with p = rho R T (Sec. IV-C) */
        t->tau_f = viscosity(g, T) / (rho * p->R * T) + 0.5;
    }
    const double sf = 1.0 / t->tau_f;
    t->s[0] = 1.0 / p->tau_rho;
    t->s[1] = p->s_e > 0.0 ? p->s_e : sf;
    t->s[2] = p->s_zeta > 0.0 ? p->s_zeta : sf;
    t->s[3] = t->s[5] = 1.0 / p->tau_j;
    t->s[4] = t->s[6] = p->s_q;
    t->s[7] = t->s[8] = sf;
    const double tau_h = (t->tau_f - 0.5) / p->Pr;
    t->omega_h = 2.0 / (2.0 * tau_h + 1.0);
    t->inv_tau_hf = (p->Pr - 1.0) / t->tau_f;
}

/* ---- moments of one node (Eq. 46, forcing note, Eq. 37 / internal form) -- */
static void moments(const orc_grid *g, const double *pp, double *rho, double *ux, double *uy, double *T) {
    double r = 0.0, jx = 0.0, jy = 0.0, sh = 0.0;
    for (int a = 0; a < NQ; ++a) {
        r += pp[a];
        jx += g->ex[a] * pp[a];
        jy += g->ey[a] * pp[a];
        sh += pp[NQ + a];
    }
    const double ax = 0.0, ay = -r * g->p.g;
    const double vx = (jx + 0.5 * ax) / r, vy = (jy + 0.5 * ay) / r;
    double t;
    if (g->p.energy == ORC_INTERNAL)
        t = 2.0 * sh / (r * g->p.b * g->p.R);
    else
        t = 2.0 / (g->p.b * g->p.R) * (sh / r - 0.5 * (vx * vx + vy * vy));
    *rho = r;
    *ux = vx;
    *uy = vy;
    *T = t;
}

/* ---- node classification ---------------------------------------------- */
enum { K_INTERIOR = 0, K_WALL, K_ADIABATIC, K_INLET, K_OUTLET, K_CORNER };

static int side_active(const orc_grid *g, int s) { return g->p.side_kind[s] != ORC_PERIODIC; }

/* Returns the node kind; for boundary nodes *fi,*fj is the node whose state is
 * extrapolated (inward normal, diagonal at corners); sx, sy name the sides hit. */
static int classify(const orc_grid *g, int i, int j, int *fi, int *fj, int *sx, int *sy) {
    int hx = -1, hy = -1;
    if (i == 0 && side_active(g, 0)) hx = 0;
    if (i == g->nx - 1 && side_active(g, 1)) hx = 1;
    if (j == 0 && side_active(g, 2)) hy = 2;
    if (j == g->ny - 1 && side_active(g, 3)) hy = 3;
    *sx = hx;
    *sy = hy;
    *fi = i;
    *fj = j;
    if (hx < 0 && hy < 0) return K_INTERIOR;
    if (hx >= 0) *fi = (hx == 0) ? 1 : g->nx - 2;
    if (hy >= 0) *fj = (hy == 2) ? 1 : g->ny - 2;
    if (hx >= 0 && hy >= 0) return K_CORNER;
    const int kind = g->p.side_kind[hx >= 0 ? hx : hy];
    switch (kind) {
    case ORC_WALL: return K_WALL;
    case ORC_ADIABATIC: return K_ADIABATIC;
    case ORC_INLET: return K_INLET;
    default: return K_OUTLET;
    }
}

/* ---- stages of a time step ---------------------------------------------- */
static size_t nid(const orc_grid *g, int i, int j) { return (size_t)j * g->nx + i; }

static void stage_moments(orc_grid *g) {
#pragma omp parallel for schedule(static) if (g->nx * g->ny >= ORC_OMP_MIN_NODES)
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) {
            const size_t k = nid(g, i, j);
            moments(g, g->pop + k * NPOP, &g->rho[k], &g->ux[k], &g->uy[k], &g->T[k]);
        }
}

static void inlet_values(const orc_grid *g, double *rho, double *ux, double *uy, double *T) {
    const orc_params *p = &g->p;
    const double gamma = (p->b + 2.0) / p->b;
    const double cs = sqrt(gamma * p->R * p->T0);
    const double s = sin(2.0 * M_PI * (double)g->n / p->side_period[0]);
    const double U0 = p->side_amp[0];
    *ux = U0 * s;
    *uy = 0.0;
    *rho = p->rho0 * (1.0 + U0 * s / cs);
    *T = p->T0 * (1.0 + (gamma - 1.0) * U0 * s / cs);
}

/* Wall density from pressure extrapolation that keeps the hydrostatic
 * balance of the body force a = (0, -rho g): p_b = p_f exp(g dy / (R T_m))
 * with dy = y_f - y_b and T_m = (T_f + T_b)/2, p = rho R T. */
static double wall_density(const orc_grid *g, double rf, double Tf, double Tb, int dy) {
    const double Tm = 0.5 * (Tf + Tb);
    return rf * Tf / Tb * exp(g->p.g * (double)dy / (g->p.R * Tm));
}

/* Boundary treatment (see the header for the readings). Reads only interior
 * nodes' populations and moments (an axis with an adiabatic wall has at least
 * four nodes, so the second node along the normal is interior too), writes
 * only boundary nodes. */
static void stage_boundary(orc_grid *g) {
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) {
            int fi, fj, sx, sy;
            const int kind = classify(g, i, j, &fi, &fj, &sx, &sy);
            if (kind == K_INTERIOR) continue;
            const size_t k = nid(g, i, j), kf = nid(g, fi, fj);
            double *pb = g->pop + k * NPOP;
            const double *pf = g->pop + kf * NPOP;
            const double rf = g->rho[kf], Tf = g->T[kf];
            double rb, uxb, uyb, Tb;
            if (kind == K_INLET) {
                inlet_values(g, &rb, &uxb, &uyb, &Tb);
                double fe[NQ], he[NQ];
                feq(g, rb, uxb, uyb, Tb, fe);
                heq(g, rb, uxb, uyb, Tb, fe, he);
                for (int a = 0; a < NQ; ++a) {
                    pb[a] = fe[a];
                    pb[NQ + a] = he[a];
                }
            } else if (kind == K_OUTLET) {
                rb = rf;
                uxb = g->ux[kf];
                uyb = g->uy[kf];
                Tb = Tf;
                for (int a = 0; a < NPOP; ++a) pb[a] = pf[a];
            } else {
                int dirichlet = 0;
                double Twall = 0.0;
                if (kind == K_CORNER) {
                    uxb = g->p.side_ux[sx];
                    uyb = g->p.side_uy[sx];
                    if (g->p.side_kind[sx] == ORC_WALL) {
                        dirichlet = 1;
                        Twall = g->p.side_T[sx];
                    } else if (g->p.side_kind[sy] == ORC_WALL) {
                        dirichlet = 1;
                        Twall = g->p.side_T[sy];
                    }
                } else {
                    const int s = sx >= 0 ? sx : sy;
                    uxb = g->p.side_ux[s];
                    uyb = g->p.side_uy[s];
                    if (kind == K_WALL) {
                        dirichlet = 1;
                        Twall = g->p.side_T[s];
                    }
                }
                if (dirichlet) {
                    Tb = Twall;
                    rb = (g->p.rho_extrap == ORC_RHO_PRESSURE) ? wall_density(g, rf, Tf, Tb, fj - j) : rf;
                } else {
                    /* adiabatic: second-order one-sided zero normal gradient,
                     * T_b = (4 T_1 - T_2)/3 along the inward normal */
                    const int di = fi - i, dj = fj - j;
                    const double T2 = g->T[nid(g, fi + di, fj + dj)];
                    Tb = (4.0 * Tf - T2) / 3.0;
                    rb = (g->p.rho_extrap == ORC_RHO_PRESSURE) ? wall_density(g, rf, Tf, Tb, fj - j) : rf;
                }
                double feb[NQ], heb[NQ], fef[NQ], hef[NQ];
                feq(g, rb, uxb, uyb, Tb, feb);
                heq(g, rb, uxb, uyb, Tb, feb, heb);
                feq(g, rf, g->ux[kf], g->uy[kf], Tf, fef);
                heq(g, rf, g->ux[kf], g->uy[kf], Tf, fef, hef);
                for (int a = 0; a < NQ; ++a) {
                    pb[a] = feb[a] + (pf[a] - fef[a]);
                    pb[NQ + a] = heb[a] + (pf[NQ + a] - hef[a]);
                }
            }
            g->rho[k] = rb;
            g->ux[k] = uxb;
            g->uy[k] = uyb;
            g->T[k] = Tb;
        }
}

/* Moments and boundary treatment of the current state. Idempotent. */
static void prepare(orc_grid *g) {
    stage_moments(g);
    stage_boundary(g);
}

static int use_correction(const orc_grid *g) { return g->p.correction && g->p.coupled; }

/* Collision of one node with given phi (Eq. 44 / Eq. 34, Eq. 47). */
static void collide_node(const orc_grid *g, const double *pin, double rho, double ux, double uy, double T,
                         double phix, double phiy, int inlet, double *pout) {
    const double *f = pin, *h = pin + NQ;
    double *fo = pout, *ho = pout + NQ;
    double fe[NQ], he[NQ];
    feq(g, rho, ux, uy, T, fe);
    heq(g, rho, ux, uy, T, fe, he);
    if (inlet) {
        for (int a = 0; a < NQ; ++a) {
            fo[a] = fe[a];
            ho[a] = he[a];
        }
        return;
    }
    transport t;
    transport_at(g, rho, T, &t);
    const double ax = 0.0, ay = -rho * g->p.g;

    /* sources: C^ = (0, phi_x, 0, 0, 0, 0, 0, phi_y, 0) + F^ and C = M^-1 C^ */
    double Chat[NQ], Fh[NQ], Cv[NQ], Fv[NQ];
    forcing_mom(ux, uy, ax, ay, Fh);
    for (int k = 0; k < NQ; ++k) Chat[k] = Fh[k];
    Chat[1] += phix;
    Chat[7] += phiy;
    correction_vel(phix, phiy, Cv);
    forcing_vel(g, ux, uy, ax, ay, Fv);
    for (int a = 0; a < NQ; ++a) Cv[a] += Fv[a];

    if (g->p.collision == ORC_MRT) {
        double m[NQ], me[NQ], ms[NQ];
        matvec9(MB1, f, m);
        meq(g, rho, ux, uy, T, me);
        for (int k = 0; k < NQ; ++k) ms[k] = m[k] - t.s[k] * (m[k] - me[k]) + (1.0 - 0.5 * t.s[k]) * Chat[k];
        matvec9(MB2, ms, fo);
    } else {
        const double wf = 1.0 / t.tau_f;
        for (int a = 0; a < NQ; ++a) fo[a] = f[a] - wf * (f[a] - fe[a]) + (1.0 - 0.5 * wf) * Cv[a];
    }

    const int heat = (g->p.energy == ORC_TOTAL) && g->p.heating;
    for (int a = 0; a < NQ; ++a) {
        double hn = h[a] - t.omega_h * (h[a] - he[a]);
        if (heat) {
            const double Z = g->ex[a] * ux + g->ey[a] * uy;
            hn += (1.0 - 0.5 * t.omega_h) * Z * t.inv_tau_hf * (f[a] - fe[a] + 0.5 * Cv[a]);
        }
        ho[a] = hn;
    }
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

static void stage_collide(orc_grid *g) {
    /* Q = rho u (1 - theta), Eq. 48 */
    for (size_t k = 0; k < (size_t)g->nx * g->ny; ++k) {
        const double th = g->T[k] / g->p.T0;
        g->Qx[k] = g->rho[k] * g->ux[k] * (1.0 - th);
        g->Qy[k] = g->rho[k] * g->uy[k] * (1.0 - th);
    }
    const int corr = use_correction(g);
#pragma omp parallel for schedule(static) if (g->nx * g->ny >= ORC_OMP_MIN_NODES)
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) {
            int fi, fj, sx, sy;
            const int kind = classify(g, i, j, &fi, &fj, &sx, &sy);
            const size_t k = nid(g, i, j);
            double phix = 0.0, phiy = 0.0;
            if (corr && kind == K_INTERIOR) {
                /* Eq. 50, second-order central differences, periodic wrap */
                const double dQx = 0.5 * (g->Qx[nid(g, wrap(i + 1, g->nx), j)] - g->Qx[nid(g, wrap(i - 1, g->nx), j)]);
                const double dQy = 0.5 * (g->Qy[nid(g, i, wrap(j + 1, g->ny))] - g->Qy[nid(g, i, wrap(j - 1, g->ny))]);
                phix = 3.0 * (dQx + dQy);
                phiy = dQx - dQy;
            }
            collide_node(g, g->pop + k * NPOP, g->rho[k], g->ux[k], g->uy[k], g->T[k], phix, phiy,
                         kind == K_INLET, g->post + k * NPOP);
        }
}

/* Eq. 45: push streaming; leaving through a non-periodic side drops the value. */
static void stage_stream(orc_grid *g) {
    const size_t n = (size_t)g->nx * g->ny * NPOP;
    for (size_t k = 0; k < n; ++k) g->pop[k] = NAN;
    const int perx = !side_active(g, 0) && !side_active(g, 1);
    const int pery = !side_active(g, 2) && !side_active(g, 3);
#pragma omp parallel for schedule(static) if (g->nx * g->ny >= ORC_OMP_MIN_NODES)
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) {
            const double *src = g->post + nid(g, i, j) * NPOP;
            for (int a = 0; a < NQ; ++a) {
                int ti = i + g->ex[a], tj = j + g->ey[a];
                if (ti < 0 || ti >= g->nx) {
                    if (!perx) continue;
                    ti = wrap(ti, g->nx);
                }
                if (tj < 0 || tj >= g->ny) {
                    if (!pery) continue;
                    tj = wrap(tj, g->ny);
                }
                double *dst = g->pop + nid(g, ti, tj) * NPOP;
                dst[a] = src[a];
                dst[NQ + a] = src[NQ + a];
            }
        }
}

/* ---- public entry points (ctypes) --------------------------------------- */
orc_grid *orc_create(const orc_params *p) {
    if (p->nx < 1 || p->ny < 1) return NULL;
    orc_grid *g = (orc_grid *)calloc(1, sizeof(orc_grid));
    g->p = *p;
    g->nx = p->nx;
    g->ny = p->ny;
    lattice(g->ex, g->ey, g->w);
    const size_t N = (size_t)p->nx * p->ny;
    g->pop = (double *)calloc(N * NPOP, sizeof(double));
    g->post = (double *)calloc(N * NPOP, sizeof(double));
    g->rho = (double *)calloc(N, sizeof(double));
    g->ux = (double *)calloc(N, sizeof(double));
    g->uy = (double *)calloc(N, sizeof(double));
    g->T = (double *)calloc(N, sizeof(double));
    g->Qx = (double *)calloc(N, sizeof(double));
    g->Qy = (double *)calloc(N, sizeof(double));
    g->Tsnap = (double *)calloc(N, sizeof(double));
    return g;
}

void orc_destroy(orc_grid *g) {
    if (!g) return;
    free(g->pop);
    free(g->post);
    free(g->rho);
    free(g->ux);
    free(g->uy);
    free(g->T);
    free(g->Qx);
    free(g->Qy);
    free(g->Tsnap);
    free(g);
}

/* Initial state: equilibria of the given fields (NULL: rho0, 0, 0, T0). */
void orc_init(orc_grid *g, const double *rho, const double *ux, const double *uy, const double *T) {
    const size_t N = (size_t)g->nx * g->ny;
    for (size_t k = 0; k < N; ++k) {
        const double r = rho ? rho[k] : g->p.rho0, vx = ux ? ux[k] : 0.0, vy = uy ? uy[k] : 0.0,
                     t = T ? T[k] : g->p.T0;
        double fe[NQ], he[NQ];
        feq(g, r, vx, vy, t, fe);
        heq(g, r, vx, vy, t, fe, he);
        for (int a = 0; a < NQ; ++a) {
            g->pop[k * NPOP + a] = fe[a];
            g->pop[k * NPOP + NQ + a] = he[a];
        }
    }
    g->n = 0;
    g->have_snap = 0;
}

void orc_step(orc_grid *g, long nsteps) {
    for (long s = 0; s < nsteps; ++s) {
        prepare(g);
        stage_collide(g);
        stage_stream(g);
        g->n += 1;
    }
}

/* Streaming only (test hook for Eq. 45). */
void orc_stream_only(orc_grid *g, long nsteps) {
    const size_t n = (size_t)g->nx * g->ny * NPOP;
    for (long s = 0; s < nsteps; ++s) {
        memcpy(g->post, g->pop, n * sizeof(double));
        stage_stream(g);
        g->n += 1;
    }
}

long orc_time(const orc_grid *g) { return g->n; }

/* Moments after the boundary treatment at the current time. */
void orc_macros(orc_grid *g, double *rho, double *ux, double *uy, double *T) {
    prepare(g);
    const size_t N = (size_t)g->nx * g->ny;
    memcpy(rho, g->rho, N * sizeof(double));
    memcpy(ux, g->ux, N * sizeof(double));
    memcpy(uy, g->uy, N * sizeof(double));
    memcpy(T, g->T, N * sizeof(double));
}

/* Pre-collision populations after the boundary treatment, [18][ny][nx]. */
void orc_pops(orc_grid *g, double *out) {
    prepare(g);
    const size_t N = (size_t)g->nx * g->ny;
    for (size_t k = 0; k < N; ++k)
        for (int a = 0; a < NPOP; ++a) out[(size_t)a * N + k] = g->pop[k * NPOP + a];
}

/* Overwrite the pre-collision populations ([18][ny][nx]). */
void orc_set_pops(orc_grid *g, const double *in) {
    const size_t N = (size_t)g->nx * g->ny;
    for (size_t k = 0; k < N; ++k)
        for (int a = 0; a < NPOP; ++a) g->pop[k * NPOP + a] = in[(size_t)a * N + k];
}

/* out = {sum f, sum h, sum e_x f, sum e_y f, #non-finite or non-positive nodes} */
void orc_diag(orc_grid *g, double *out) {
    prepare(g);
    double m = 0.0, e = 0.0, jx = 0.0, jy = 0.0, bad = 0.0;
    const size_t N = (size_t)g->nx * g->ny;
    for (size_t k = 0; k < N; ++k) {
        const double *pp = g->pop + k * NPOP;
        for (int a = 0; a < NQ; ++a) {
            m += pp[a];
            e += pp[NQ + a];
            jx += g->ex[a] * pp[a];
            jy += g->ey[a] * pp[a];
        }
        if (!(isfinite(g->rho[k]) && isfinite(g->ux[k]) && isfinite(g->uy[k]) && isfinite(g->T[k]) &&
              g->rho[k] > 0.0 && g->T[k] > 0.0))
            bad += 1.0;
    }
    out[0] = m;
    out[1] = e;
    out[2] = jx;
    out[3] = jy;
    out[4] = bad;
}

/* r = ||T - T_snap||_2 / ||T||_2 against the previous snapshot (inf on the
 * first call); when update != 0 the snapshot becomes the current T. */
double orc_residual(orc_grid *g, int update) {
    prepare(g);
    const size_t N = (size_t)g->nx * g->ny;
    double num = 0.0, den = 0.0;
    for (size_t k = 0; k < N; ++k) {
        const double d = g->T[k] - g->Tsnap[k];
        num += d * d;
        den += g->T[k] * g->T[k];
    }
    const double r = g->have_snap ? sqrt(num) / sqrt(den) : INFINITY;
    if (update) {
        memcpy(g->Tsnap, g->T, N * sizeof(double));
        g->have_snap = 1;
    }
    return r;
}

/* Threads of the OpenMP passes (timing of the CPU baseline); ignored without
 * OpenMP. */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---- single-node entry points used by the pins ------------------------- */
void orc_lattice(int *ex, int *ey, double *w) { lattice(ex, ey, w); }

void orc_matrices(double *M, double *Minv) {
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) {
            M[r * 9 + c] = MB1[r][c];
            Minv[r * 9 + c] = MB2[r][c];
        }
}

void orc_node_feq(const orc_grid *g, double rho, double ux, double uy, double T, double *out) {
    feq(g, rho, ux, uy, T, out);
}

void orc_node_heq(const orc_grid *g, double rho, double ux, double uy, double T, double *out) {
    double fe[NQ];
    feq(g, rho, ux, uy, T, fe);
    heq(g, rho, ux, uy, T, fe, out);
}

void orc_node_meq(const orc_grid *g, double rho, double ux, double uy, double T, double *out) {
    meq(g, rho, ux, uy, T, out);
}

void orc_node_correction(double phix, double phiy, double *out) { correction_vel(phix, phiy, out); }

void orc_node_forcing(const orc_grid *g, double ux, double uy, double ax, double ay, double *Fv, double *Fh) {
    forcing_vel(g, ux, uy, ax, ay, Fv);
    forcing_mom(ux, uy, ax, ay, Fh);
}

void orc_node_moments(const orc_grid *g, const double *pin, double *out4) {
    moments(g, pin, &out4[0], &out4[1], &out4[2], &out4[3]);
}

/* Collide one interior node with the given gradients: pin/pout hold 18 values. */
void orc_node_collide(const orc_grid *g, const double *pin, double phix, double phiy, double *pout) {
    double r, vx, vy, t;
    moments(g, pin, &r, &vx, &vy, &t);
    collide_node(g, pin, r, vx, vy, t, phix, phiy, 0, pout);
}

void orc_node_transport(const orc_grid *g, double rho, double T, double *out12) {
    transport t;
    transport_at(g, rho, T, &t);
    out12[0] = t.tau_f;
    for (int k = 0; k < NQ; ++k) out12[1 + k] = t.s[k];
    out12[10] = t.omega_h;
    out12[11] = t.inv_tau_hf;
}
