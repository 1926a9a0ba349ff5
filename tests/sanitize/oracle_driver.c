/* The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: every
 * flag of the step on small grids (plates and periodic, odd sizes, the
 * smallest grids the open ends and the plates allow), the EOS helpers and
 * the exported right-hand side of the energy equation.  Test
 * infrastructure: tests/test_sanitizers.py compiles this file (which
 * includes the oracle's source) with -fsanitize=address,undefined and runs
 * it; any report aborts the run. */
#include "../../oracle/lbm_oracle.c"

#include <stdio.h>

static orc_params base(int Nx, int Ny, uint32_t flags) {
    orc_params p;
    memset(&p, 0, sizeof(p));
    p.Nx = Nx;
    p.Ny = Ny;
    p.flags = flags;
    double rc;
    if (flags & ORC_EOS_CS) {
        p.a = 1.0, p.b = 4.0, p.R = 1.0;
        orc_critical_cs(p.a, p.b, p.R, &rc, &p.Tc);
        p.lambda = 0.05;
    } else {
        p.a = 3.0 / 49.0, p.b = 2.0 / 21.0, p.R = 1.0, p.omega = 0.344;
        orc_critical(p.a, p.b, p.R, &rc, &p.Tc);
        p.lambda = 0.25;
    }
    p.G = -1.0, p.theta = 0.104;
    p.s_rho = 1.0, p.s_e = p.s_zeta = 0.8, p.s_j = 1.0, p.s_q = 1.1;
    p.tau_g = 0.8, p.tau_l = 1.3;
    p.Cv = 5.0;
    p.T0 = 0.86 * p.Tc, p.Tw = 0.78 * p.Tc;
    p.g_osc = 1e-4, p.period = 50.0;
    double ps;
    orc_maxwell(&p, p.T0, &p.rho_g, &p.rho_l, &ps);
    p.rho_v = p.rho_g;
    p.Gw = p.G;
    p.psiw = orc_psi(&p, 0.5 * (p.rho_g + p.rho_l), p.T0);
    if (flags & ORC_FRAME_RHO) p.rho_frame = 0.9 * p.rho_g;
    if (flags & ORC_OPEN_X) {
        p.g_osc = 0.0, p.gx = 1e-4;
        p.p_amp = 0.1, p.p_period = 40.0;
        p.Tw = 0.86 * p.Tc, p.Tw_end = 0.56 * p.Tc, p.T_in = p.T0, p.T_out = p.T0;
        p.alpha_max = 0.25;
    }
    if (flags & ORC_PHASE_PROPS) p.lam_l = 0.6, p.Cv_l = 3.0;
    if (flags & ORC_TOP_MIXED) p.cold_x0 = Nx / 3, p.cold_x1 = 2 * Nx / 3, p.Tw_bot = p.T0;
    return p;
}

/* a liquid layer on the lower plate with a deterministic ripple (vapour
 * only with open ends, whose columns take vapour densities) */
static void layer(const orc_params* p, double* rho) {
    for (int y = 0; y < p->Ny; ++y)
        for (int x = 0; x < p->Nx; ++x) {
            double h = (p->flags & ORC_OPEN_X) ? 0.0 : 0.5 * (1.0 - tanh((y - p->Ny / 3.0) / 1.5));
            double r = p->rho_g + (p->rho_l - p->rho_g) * h;
            rho[(size_t)y * p->Nx + x] = r * (1.0 + 0.01 * sin(1.7 * x + 0.3 * y));
        }
}

static int run(orc_params p, int steps) {
    const size_t N = (size_t)p.Nx * p.Ny;
    double* rho = (double*)malloc(6 * N * sizeof(double));
    double *ux = rho + N, *uy = rho + 2 * N, *T = rho + 3 * N, *Fx = rho + 4 * N, *Fy = rho + 5 * N;
    double* K = (double*)malloc(N * sizeof(double));
    layer(&p, rho);
    orc_sim* s = orc_sim_new(&p);
    if (!s) return 1;
    orc_sim_init(s, rho, 0.0);
    orc_sim_step(s, steps);
    orc_sim_moments(s, rho, ux, uy, T, Fx, Fy);
    orc_heat_rhs(&p, rho, ux, uy, T, K);
    double acc = 0.0;
    for (size_t c = 0; c < N; ++c) acc += rho[c] + T[c] + K[c];
    double* f = (double*)malloc(9 * N * sizeof(double));
    orc_sim_get_f(s, f);
    orc_sim_set_f(s, f);
    orc_sim_set_T(s, T);
    orc_sim_step(s, 1);
    free(f);
    orc_sim_free(s);
    free(rho);
    free(K);
    return !(acc == acc);  /* finite */
}

int main(void) {
    const uint32_t flag_sets[] = {
        0, ORC_FREEZE_T, ORC_SINGLE_PHASE, ORC_PERIODIC_Y, ORC_FRAME_T,
        ORC_FRAME_T | ORC_PERIODIC_Y, ORC_FRAME_RHO, ORC_FRAME_T | ORC_FRAME_RHO | ORC_PERIODIC_Y,
        ORC_EOS_CS, ORC_OPEN_X, ORC_OPEN_X | ORC_PHASE_PROPS, ORC_PHASE_PROPS, ORC_TOP_MIXED,
        ORC_TOP_MIXED | ORC_PHASE_PROPS};
    const int grids[][2] = {{13, 9}, {4, 4}, {6, 3}, {9, 17}};
    int runs = 0, bad = 0;
    for (size_t k = 0; k < sizeof(flag_sets) / sizeof(flag_sets[0]); ++k)
        for (size_t g = 0; g < sizeof(grids) / sizeof(grids[0]); ++g) {
            const uint32_t fl = flag_sets[k];
            const int Nx = grids[g][0], Ny = grids[g][1];
            if (!(fl & ORC_PERIODIC_Y) && Ny < 3) continue;
            orc_params p = base(Nx, Ny, fl);
            const int nb = run(p, 12);
            if (nb) printf("non-finite: flags %u grid %dx%d\n", fl, Nx, Ny);
            bad += nb;
            ++runs;
        }
    /* EOS helpers over a temperature range */
    orc_params p = base(8, 8, 0);
    for (double t = 0.55; t < 0.99; t += 0.04) {
        double g, l, ps, h;
        orc_maxwell(&p, t * p.Tc, &g, &l, &ps);
        orc_latent_heat(&p, t * p.Tc, &h);
    }
    orc_params q = base(16, 8, ORC_OPEN_X);
    for (int64_t n = 0; n < 40; ++n) (void)orc_inlet_density(&q, n);
    printf("oracle sanitizer runs: %d configurations, %d non-finite\n", runs, bad);
    return bad != 0;
}
