/* The host side of the runtime under AddressSanitizer and
 * UndefinedBehaviorSanitizer, through the C-ABI of include/lbm.h.
 *
 * Without arguments: the entry points that run on the host only (parameter
 * defaults and derivation, every validation rule, the EOS helpers, the
 * footprint and workspace sizes, the initial-density checks, null and
 * invalid arguments); lbm_create and lbm_pool_create are called too and end
 * at their first device call when there is no GPU.
 * With "gpu": also a simulation (steps, moments, reductions, checkpoint
 * round trip, launch shapes, autotune) and a pool (admission under a cap,
 * chunks, poll, read-out, health, release and reuse of slots, autotune),
 * which exercises the host-side bookkeeping with real device work.
 *
 * Test infrastructure: tests/test_sanitizers.py links this file against a
 * build of the library whose host code carries the sanitizers. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#include <unistd.h>

#include "lbm.h"

static int failures = 0;
#define EXPECT(cond)                                                          \
    do {                                                                      \
        if (!(cond)) {                                                        \
            fprintf(stderr, "%s:%d: expectation failed: %s (%s)\n", __FILE__, \
                    __LINE__, #cond, lbm_last_error());                       \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

static lbm_params channel(int Nx, int Ny, uint32_t flags) {
    lbm_params p;
    lbm_params_default(&p);
    p.Nx = Nx;
    p.Ny = Ny;
    p.flags = flags;
    if (flags & LBM_EOS_CS) {
        p.a = 1.0, p.b = 4.0, p.R = 1.0, p.lambda = 0.05;
    }
    EXPECT(lbm_params_resolve(&p) == LBM_OK);
    double P, psi;
    EXPECT(lbm_eos_pressure(&p, 0.5 * (p.rho_g + p.rho_l), p.T_0, &P, &psi) == LBM_OK);
    p.G_w = p.G;
    p.psi_w = psi;
    if (flags & LBM_FRAME_RHO) p.rho_frame = 0.9 * p.rho_g;
    if (flags & LBM_OPEN_X) {
        p.g_osc = 0.0, p.g_x = 1e-4, p.p_amp = 0.1, p.p_period = 40.0;
        p.T_w = 0.86 * p.T_c, p.T_w_end = 0.56 * p.T_c, p.T_in = p.T_0, p.T_out = p.T_0;
        p.alpha_max = 0.25;
    }
    if (flags & LBM_PHASE_PROPS) p.lambda_l = 0.6, p.C_v_l = 3.0;
    if (flags & LBM_TOP_MIXED) p.cold_x0 = Nx / 3, p.cold_x1 = 2 * Nx / 3;
    return p;
}

static double* vapour(const lbm_params* p) {
    double* r = (double*)malloc((size_t)p->Nx * p->Ny * sizeof(double));
    for (int y = 0; y < p->Ny; ++y)
        for (int x = 0; x < p->Nx; ++x)
            r[(size_t)y * p->Nx + x] = p->rho_v * (1.0 + 0.01 * sin(0.7 * x + 1.3 * y));
    return r;
}

static void host_only(void) {
    double rc, tc, g, l, ps, h, ja, P, psi;
    EXPECT(lbm_eos_critical(3.0 / 49.0, 2.0 / 21.0, 1.0, &rc, &tc) == LBM_OK);
    EXPECT(lbm_eos_critical_cs(1.0, 4.0, 1.0, &rc, &tc) == LBM_OK);
    EXPECT(lbm_eos_critical(-1.0, 1.0, 1.0, &rc, &tc) == LBM_EINVAL);
    EXPECT(lbm_eos_critical(1.0, 1.0, 1.0, NULL, &tc) == LBM_EINVAL);
    lbm_params p = channel(64, 20, 0);
    for (double t = 0.5; t < 1.0; t += 0.03) {
        (void)lbm_eos_coexistence(&p, t * p.T_c, &g, &l, &ps);
        (void)lbm_eos_latent_heat(&p, t * p.T_c, &h);
        (void)lbm_eos_jacob(&p, p.T_0, t * p.T_c, &ja);
        (void)lbm_eos_pressure(&p, 1.0 + 8.0 * t, t * p.T_c, &P, &psi);
    }
    EXPECT(lbm_eos_coexistence(&p, 1.2 * p.T_c, &g, &l, &ps) != LBM_OK);
    EXPECT(lbm_eos_pressure(NULL, 1.0, 1.0, &P, &psi) == LBM_EINVAL);
    const uint32_t flag_sets[] = {0, LBM_FREEZE_T, LBM_SINGLE_PHASE, LBM_PERIODIC_Y, LBM_FRAME_T,
                                  LBM_FRAME_RHO, LBM_EOS_CS, LBM_OPEN_X,
                                  LBM_OPEN_X | LBM_PHASE_PROPS, LBM_PHASE_PROPS, LBM_TOP_MIXED};
    for (size_t k = 0; k < sizeof(flag_sets) / sizeof(flag_sets[0]); ++k) {
        lbm_params q = channel(70, 24, flag_sets[k]);
        EXPECT(lbm_workspace_bytes(&q) > 0);
        EXPECT(lbm_pool_footprint(&q) > 0);
    }
    /* every validation rule refuses */
    lbm_params bad[16];
    int nb = 0;
    bad[nb] = p, bad[nb++].Nx = 2;
    bad[nb] = p, bad[nb++].Ny = 3;
    bad[nb] = p, bad[nb++].precision = 7;
    bad[nb] = p, bad[nb++].flags = 1u << 12;
    bad[nb] = p, bad[nb++].s_e = 0.9;
    bad[nb] = p, bad[nb++].tau_g = 0.5;
    bad[nb] = p, bad[nb++].G = 0.0;
    bad[nb] = p, bad[nb++].alpha_max = 0.6;
    bad[nb] = p, bad[nb++].T_out = 0.5;  /* without LBM_OPEN_X */
    bad[nb] = p, bad[nb].flags = LBM_TOP_MIXED | LBM_OPEN_X, ++nb;
    bad[nb] = p, bad[nb].flags = LBM_PHASE_PROPS, bad[nb++].C_v_l = 0.0;
    bad[nb] = p, bad[nb].flags = LBM_FRAME_RHO, bad[nb++].rho_frame = 0.0;
    bad[nb] = p, bad[nb++].Nx = 1 << 22;  /* buffers beyond 32-bit offsets */
    for (int k = 0; k < nb; ++k) {
        EXPECT(lbm_workspace_bytes(&bad[k]) == 0);
        EXPECT(lbm_pool_footprint(&bad[k]) == 0);
        lbm_sim* s = NULL;
        EXPECT(lbm_create(&bad[k], NULL, NULL, 0, NULL, &s) == LBM_EINVAL && s == NULL);
        EXPECT(strlen(lbm_last_error()) > 0);
    }
    /* initial densities outside the EOS range or without a real psi */
    double* r = vapour(&p);
    r[5 * p.Nx + 7] = -1.0;
    lbm_sim* s = NULL;
    EXPECT(lbm_create(&p, r, NULL, 0, NULL, &s) == LBM_EINVAL);
    r[5 * p.Nx + 7] = 9.6;
    EXPECT(lbm_create(&p, r, NULL, 0, NULL, &s) == LBM_EINVAL);
    free(r);
    /* null arguments */
    EXPECT(lbm_create(NULL, NULL, NULL, 0, NULL, &s) == LBM_EINVAL);
    EXPECT(lbm_create(&p, NULL, NULL, 0, NULL, NULL) == LBM_EINVAL);
    EXPECT(lbm_step(NULL, 1) == LBM_EINVAL);
    EXPECT(lbm_moments(NULL, NULL, NULL, NULL, NULL) == LBM_EINVAL);
    EXPECT(lbm_destroy(NULL) == LBM_OK);
    EXPECT(lbm_pool_destroy(NULL) == LBM_OK);
    EXPECT(lbm_pool_footprint(NULL) == 0);
    EXPECT(lbm_pool_run(NULL, 1) == LBM_EINVAL);
    EXPECT(lbm_pool_autotune(NULL, 1, NULL) == LBM_EINVAL);
    EXPECT(lbm_pool_slot_time(NULL, 0) == -1);
}

/* Random parameter sets (a fixed xorshift sequence): every double field may
 * become zero, negative, huge, infinite or NaN, every integer field an edge
 * value; the host-only entry points must return a status or a size. */
static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static uint64_t next_u64(void) {
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return rng_state;
}
static void fuzz_params(int rounds) {
    const double special[] = {0.0, -1.0, 1e300, -1e300, INFINITY, -INFINITY, NAN, 1e-300, 0.5, 2.0};
    const int32_t ints[] = {0, -1, 1, 2, 3, 4, 5, 64, 1 << 20, INT32_MIN, INT32_MAX};
    const lbm_params base = channel(96, 24, 0);
    for (int r = 0; r < rounds; ++r) {
        lbm_params p = base;
        double* d = &p.a;  /* the doubles from a to rho_frame... are contiguous in groups */
        (void)d;
        unsigned char* raw = (unsigned char*)&p;
        /* walk the struct field by field through known offsets */
        const size_t dbl_first = offsetof(lbm_params, a), dbl_last = offsetof(lbm_params, T_w_bottom);
        for (size_t o = dbl_first; o <= dbl_last; o += sizeof(double))
            if (next_u64() % 8 == 0) {
                double v = special[next_u64() % (sizeof(special) / sizeof(special[0]))];
                memcpy(raw + o, &v, sizeof(v));
            }
        if (next_u64() % 8 == 0) p.Nx = ints[next_u64() % 11];
        if (next_u64() % 8 == 0) p.Ny = ints[next_u64() % 11];
        if (next_u64() % 8 == 0) p.cold_x0 = ints[next_u64() % 11];
        if (next_u64() % 8 == 0) p.cold_x1 = ints[next_u64() % 11];
        if (next_u64() % 8 == 0) p.precision = ints[next_u64() % 11];
        if (next_u64() % 4 == 0) p.flags = (uint32_t)(next_u64() % 1024);
        if (next_u64() % 8 == 0) p.alpha_max = special[next_u64() % 10];
        if (next_u64() % 8 == 0) p.T_out = special[next_u64() % 10];
        lbm_params q = p;
        (void)lbm_params_resolve(&q);
        const size_t ws = lbm_workspace_bytes(&p);
        (void)lbm_pool_footprint(&p);
        double g, l, ps, h;
        (void)lbm_eos_coexistence(&p, base.T_0, &g, &l, &ps);
        (void)lbm_eos_latent_heat(&p, base.T_0, &h);
        if (ws > 0 && p.Nx <= 4096 && p.Ny <= 4096) {
            lbm_sim* s = NULL;
            const lbm_status st = lbm_create(&p, NULL, NULL, 0, NULL, &s);
            if (st == LBM_OK) lbm_destroy(s);
        }
    }
}

static void with_gpu(void) {
    const uint32_t flag_sets[] = {0, LBM_PERIODIC_Y, LBM_OPEN_X, LBM_PHASE_PROPS, LBM_TOP_MIXED};
    for (size_t k = 0; k < sizeof(flag_sets) / sizeof(flag_sets[0]); ++k)
        for (int prec = LBM_FP32_DEV; prec <= LBM_FP32_DEV_MASSEXACT; ++prec) {
            lbm_params p = channel(130, 24, flag_sets[k]);
            p.precision = prec;
            double* r = vapour(&p);
            lbm_sim* s = NULL;
            EXPECT(lbm_create(&p, r, NULL, 0, NULL, &s) == LBM_OK);
            if (!s) {
                free(r);
                continue;
            }
            EXPECT(lbm_step(s, 13) == LBM_OK);
            const size_t N = (size_t)p.Nx * p.Ny;
            double* m = (double*)malloc(4 * N * sizeof(double));
            EXPECT(lbm_moments(s, m, m + N, m + 2 * N, m + 3 * N) == LBM_OK);
            double red[5];
            EXPECT(lbm_reduce(s, red) == LBM_OK);
            int64_t nf = -1, cl = -1;
            EXPECT(lbm_health(s, &nf, &cl) == LBM_OK && nf == 0);
            const size_t nbytes = lbm_state_bytes(s);
            char* blob = (char*)malloc(nbytes);
            EXPECT(lbm_save(s, blob, nbytes) == LBM_OK);
            EXPECT(lbm_step(s, 3) == LBM_OK);
            EXPECT(lbm_load(s, blob, nbytes) == LBM_OK && lbm_time(s) == 13);
            EXPECT(lbm_load(s, blob, nbytes - 1) == LBM_EINVAL);
            EXPECT(lbm_set_launch(s, 8) == LBM_OK);
            int32_t sr = 0, waves = 0;
            EXPECT(lbm_get_launch(s, &sr, &waves) == LBM_OK && sr == 8);
            double best = 0.0;
            EXPECT(lbm_autotune(s, 2, &best) == LBM_OK && best > 0.0);
            lbm_params got;
            EXPECT(lbm_get_params(s, &got) == LBM_OK && got.Nx == p.Nx);
            EXPECT(lbm_synchronize(s) == LBM_OK);
            EXPECT(lbm_destroy(s) == LBM_OK);
            free(blob);
            free(m);
            free(r);
        }
    /* a pool under a cap that admits about three of the channels at once */
    lbm_params ps[7];
    for (int k = 0; k < 7; ++k) ps[k] = channel(100 + 37 * k, 20 + 8 * k, k == 3 ? LBM_OPEN_X : 0);
    lbm_pool* pool = NULL;
    EXPECT(lbm_pool_create(3 * lbm_pool_footprint(&ps[6]), NULL, &pool) == LBM_OK);
    if (!pool) return;
    int admitted = 0, finished = 0, tuned = 0;
    int32_t slots[7];
    int64_t steps[7];
    for (int k = 0; k < 7; ++k) steps[k] = 30 + 11 * k;
    /* bounded: every iteration runs a chunk of 16 steps, and no request
     * needs more than 100 steps once admitted */
    for (int iter = 0; finished < 7 && iter < 1000; ++iter) {
        while (admitted < 7) {
            double* r = vapour(&ps[admitted]);
            int32_t id = -1;
            const lbm_status st = lbm_pool_admit(pool, &ps[admitted], r, steps[admitted], &id);
            free(r);
            if (st == LBM_ENOMEM) break;
            EXPECT(st == LBM_OK);
            if (st != LBM_OK) ++finished;  /* refused: nothing to wait for */
            slots[admitted++] = st == LBM_OK ? id : -2;
        }
        if (!tuned && admitted >= 3) {
            double best = 0.0;
            EXPECT(lbm_pool_autotune(pool, 2, &best) == LBM_OK && best > 0.0);
            int32_t sr = 0, w = 0;
            EXPECT(lbm_pool_slot_launch(pool, slots[0], &sr, &w) == LBM_OK && w > 0);
            tuned = 1;
        }
        EXPECT(lbm_pool_run(pool, 16) == LBM_OK);
        EXPECT(lbm_pool_wait(pool, 1) == LBM_OK);
        int32_t done[8], nd = 0;
        EXPECT(lbm_pool_poll(pool, done, 8, &nd) == LBM_OK);
        for (int i = 0; i < nd; ++i) {
            int k = 0;
            while (k < admitted && slots[k] != done[i]) ++k;
            const size_t N = (size_t)ps[k].Nx * ps[k].Ny;
            double* m = (double*)malloc(4 * N * sizeof(double));
            EXPECT(lbm_pool_moments(pool, done[i], m, m + N, m + 2 * N, m + 3 * N) == LBM_OK);
            int64_t nf = -1, cl = -1;
            EXPECT(lbm_pool_slot_health(pool, done[i], &nf, &cl) == LBM_OK && nf == 0);
            EXPECT(lbm_pool_slot_time(pool, done[i]) == steps[k]);
            EXPECT(lbm_pool_release(pool, done[i]) == LBM_OK);
            slots[k] = -2;
            free(m);
            ++finished;
        }
        EXPECT(nd >= 0);
    }
    EXPECT(finished == 7);
    int32_t active = -1;
    size_t used = 1, cap = 0;
    EXPECT(lbm_pool_info(pool, &active, &used, &cap) == LBM_OK && active == 0 && used == 0);
    EXPECT(lbm_pool_synchronize(pool) == LBM_OK);
    EXPECT(lbm_pool_destroy(pool) == LBM_OK);
}

/* Random sequences of pool operations with the GPU: admissions of small
 * channels (some with the optional features, some that turn non-finite and
 * are retired) under a cap that binds, chunks of random length, read-outs,
 * releases of finished and of unfinished slots, tuning and launch-shape
 * changes.  Checks the bookkeeping: bytes in use equal the footprints held,
 * no slot passes its step count, finished healthy slots read out with
 * LBM_OK and retired ones with LBM_EUNSTABLE.  Bounded: at most `rounds`
 * operations, then the pool is drained (every slot holds at most 60
 * steps). */
static void fuzz_pool(int rounds) {
    enum { kMax = 64 };
    lbm_params ps[kMax];
    int hot[kMax];
    size_t held[kMax];
    int32_t slot_of[kMax];
    int n = 0;
    lbm_pool* pool = NULL;
    const lbm_params big = channel(200, 40, 0);
    EXPECT(lbm_pool_create(4 * lbm_pool_footprint(&big), NULL, &pool) == LBM_OK);
    if (!pool) return;
    size_t used_expect = 0;
    int finite_ok = 0;
    for (int r = 0; r < rounds; ++r) {
        const unsigned op = (unsigned)(next_u64() % 10);
        if (op < 3 && n < kMax) {  /* admit */
            const int Nx = 20 + (int)(next_u64() % 181), Ny = 6 + (int)(next_u64() % 35);
            const uint32_t fsel[] = {0, 0, 0, LBM_OPEN_X, LBM_PHASE_PROPS, LBM_PERIODIC_Y};
            const int is_hot = (next_u64() % 8) == 0;
            lbm_params p = channel(Nx, Ny, is_hot ? 0u : fsel[next_u64() % 6]);
            if (is_hot)  /* dense supercritical fluid between hot plates */
                p.T_0 = 1.15 * p.T_c, p.T_w = 1.6 * p.T_c, p.rho_v = 7.8, p.rho_ref = 7.8;
            int32_t id = -1;
            const lbm_status st = lbm_pool_admit(pool, &p, NULL, 1 + (int64_t)(next_u64() % 60), &id);
            EXPECT(st == LBM_OK || st == LBM_ENOMEM);
            if (st == LBM_OK) {
                ps[n] = p;
                hot[n] = is_hot;
                held[n] = lbm_pool_footprint(&p);
                slot_of[n] = id;
                used_expect += held[n];
                ++n;
            }
        } else if (op < 7) {
            EXPECT(lbm_pool_run(pool, 1 + (int32_t)(next_u64() % 20)) == LBM_OK);
            EXPECT(lbm_pool_wait(pool, (int32_t)(next_u64() % 3)) == LBM_OK);
        } else if (op < 9 && n > 0) {  /* poll, read out and release what finished */
            int32_t done[kMax], nd = 0;
            EXPECT(lbm_pool_poll(pool, done, kMax, &nd) == LBM_OK);
            for (int i = 0; i < nd; ++i) {
                int k = 0;
                while (k < n && slot_of[k] != done[i]) ++k;
                if (k == n) {
                    ++failures;
                    continue;
                }
                const size_t N = (size_t)ps[k].Nx * ps[k].Ny;
                double* m = (double*)malloc(4 * N * sizeof(double));
                const lbm_status st = lbm_pool_moments(pool, done[i], m, m + N, m + 2 * N, m + 3 * N);
                /* the hot channels turn non-finite, and so can the thinnest
                 * channels: with four or five fluid rows the wall adhesion
                 * draws the vapour out of the middle rows (the oracle takes
                 * the same path, to rounding, until rho there is ~6e-4 and
                 * lambda / (rho C_v) far exceeds the RK4 bound).  The
                 * read-out status must agree with the slot's health counters
                 * either way, and wider channels must stay finite. */
                int64_t nf = -1, cl = -1;
                EXPECT(lbm_pool_slot_health(pool, done[i], &nf, &cl) == LBM_OK);
                EXPECT((st == LBM_OK && nf == 0) || (st == LBM_EUNSTABLE && nf > 0));
                if (!hot[k] && ps[k].Ny >= 12 && !(ps[k].flags & LBM_PHASE_PROPS)) {
                    EXPECT(st == LBM_OK);
                    if (st != LBM_OK)
                        fprintf(stderr, "  channel %d x %d, flags %u, n %lld\n", ps[k].Nx, ps[k].Ny,
                                ps[k].flags, (long long)lbm_pool_slot_time(pool, done[i]));
                }
                finite_ok += st == LBM_OK;
                free(m);
                EXPECT(lbm_pool_release(pool, done[i]) == LBM_OK);
                used_expect -= held[k];
                ps[k] = ps[n - 1], hot[k] = hot[n - 1], held[k] = held[n - 1];
                slot_of[k] = slot_of[n - 1];
                --n;
            }
        } else if (n > 0) {  /* release an unfinished slot, or retune */
            if (next_u64() % 2) {
                const int k = (int)(next_u64() % (uint64_t)n);
                EXPECT(lbm_pool_release(pool, slot_of[k]) == LBM_OK);
                used_expect -= held[k];
                ps[k] = ps[n - 1], hot[k] = hot[n - 1], held[k] = held[n - 1];
                slot_of[k] = slot_of[n - 1];
                --n;
            } else if (next_u64() % 2) {
                double best = 0.0;
                const lbm_status st = lbm_pool_autotune(pool, 1, &best);
                EXPECT(st == LBM_OK || st == LBM_EINVAL);
            } else {
                EXPECT(lbm_pool_set_launch(pool, (int32_t)(next_u64() % 30)) == LBM_OK);
            }
        }
        int32_t active = -1;
        size_t used = 0, cap = 0;
        EXPECT(lbm_pool_info(pool, &active, &used, &cap) == LBM_OK);
        EXPECT(active == n && used == used_expect && used <= cap);
    }
    /* drain: every remaining slot finishes within 60 steps */
    for (int it = 0; it < 8 && n > 0; ++it) {
        EXPECT(lbm_pool_run(pool, 20) == LBM_OK);
        EXPECT(lbm_pool_wait(pool, 0) == LBM_OK);
    }
    int32_t done[kMax], nd = 0;
    EXPECT(lbm_pool_poll(pool, done, kMax, &nd) == LBM_OK);
    EXPECT(nd == n);
    EXPECT(finite_ok > 0);
    EXPECT(lbm_pool_synchronize(pool) == LBM_OK);
    EXPECT(lbm_pool_destroy(pool) == LBM_OK);
}

int main(int argc, char** argv) {
    host_only();
    fuzz_params(3000);
    if (argc > 1 && strcmp(argv[1], "gpu") == 0) {
        with_gpu();
        fuzz_pool(400);
        /* end without the runtime's exit-time teardown, where the sanitizer
         * runtime's own device allocator trips over the unloaded HSA
         * runtime after main has returned */
        printf("host sanitizer driver: %d failed expectations\n", failures);
        fflush(stdout);
        fflush(stderr);
        _exit(failures != 0);
    }
    printf("host sanitizer driver: %d failed expectations\n", failures);
    return failures != 0;
}
