// Host runtime of the C-ABI declared in include/lbm.h: parameter resolution
// (Peng-Robinson critical point and coexistence, Eq. 11), memory layout,
// launch shapes, the step loop, moments, reductions and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

#include "lbm.h"
#include "lbm_host.h"
#include "lbm_internal.h"

using lbmk::Grid;
using lbmk::Phys;
using lbmhost::Layout;
using lbmhost::fail;

namespace {
thread_local char g_err[512] = "no error";
}

namespace lbmhost {

lbm_status fail(lbm_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

}  // namespace lbmhost

namespace {

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(LBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

// ---- Peng-Robinson thermodynamics (Eq. 11), host FP64 -------------------
double kappa_of(double omega) { return 0.37464 + 1.54226 * omega - 0.26992 * omega * omega; }

// With cs set, the Carnahan-Starling EOS (eta = b rho / 4):
//   P = rho R T (1 + eta + eta^2 - eta^3) / (1 - eta)^3 - a rho^2.
struct Eos {
    double a, b, R, k, Tc;
    bool cs = false;
    double phi(double T) const {
        const double s = 1.0 + k * (1.0 - std::sqrt(T / Tc));
        return s * s;
    }
    double rmax() const { return cs ? 4.0 / b : 1.0 / b; }  // packing limit
    double P(double r, double T) const {
        const double br = b * r;
        if (cs) {
            const double e = 0.25 * br, o = 1.0 - e;
            return r * R * T * (1.0 + e * (1.0 + e * (1.0 - e))) / (o * o * o) - a * r * r;
        }
        return r * R * T / (1.0 - br) - a * phi(T) * r * r / (1.0 + 2.0 * br - br * br);
    }
    double dPdr(double r, double T) const {
        const double br = b * r, D = 1.0 + 2.0 * br - br * br;
        if (cs) {
            const double e = 0.25 * br, o = 1.0 - e, o2 = o * o;
            return R * T * (1.0 + e * (4.0 + e * (4.0 + e * (-4.0 + e)))) / (o2 * o2) -
                   2.0 * a * r;
        }
        return R * T / ((1.0 - br) * (1.0 - br)) - 2.0 * a * phi(T) * r * (1.0 + br) / (D * D);
    }
    // chemical potential from the Helmholtz free energy of Eq. 11:
    // f = rho R T [ln(rho/(1 - b rho)) - 1]
    //     - a phi rho / (2 sqrt2 b) ln[(1 + (1+sqrt2) b rho) / (1 + (1-sqrt2) b rho)],
    // mu = df/drho (the additive constant drops out of equalities)
    // CS: f = rho R T [ln rho - 1 + (4 eta - 3 eta^2)/(1 - eta)^2] - a rho^2
    double mu(double r, double T) const {
        if (cs) {
            const double e = 0.25 * b * r, o = 1.0 - e;
            return R * T * (std::log(r) + e * (8.0 + e * (-9.0 + 3.0 * e)) / (o * o * o)) -
                   2.0 * a * r;
        }
        const double br = b * r, s2 = std::sqrt(2.0);
        const double L = std::log((1.0 + (1.0 + s2) * br) / (1.0 + (1.0 - s2) * br));
        return R * T * (std::log(r / (1.0 - br)) + br / (1.0 - br)) -
               a * phi(T) / (2.0 * s2 * b) * L - a * phi(T) * r / (1.0 + 2.0 * br - br * br);
    }
};

// Critical point: on the spinodal (dP/drho = 0, phi = 1) T(eta), eta = b rho,
// is proportional to eta (1+eta)(1-eta)^2 / (1+2eta-eta^2)^2; its maximum is
// the zero of the logarithmic derivative, found by bisection.
void critical_point(double a, double b, double R, double* rho_c, double* T_c) {
    auto dlog = [](double e) {
        return 1.0 / e + 1.0 / (1.0 + e) - 2.0 / (1.0 - e) -
               2.0 * (2.0 - 2.0 * e) / (1.0 + 2.0 * e - e * e);
    };
    double lo = 1e-6, hi = 1.0 - 1e-6;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (dlog(mid) > 0.0) lo = mid; else hi = mid;
    }
    const double e = 0.5 * (lo + hi), D = 1.0 + 2.0 * e - e * e;
    *rho_c = e / b;
    *T_c = 2.0 * a / (b * R) * e * (1.0 + e) * (1.0 - e) * (1.0 - e) / (D * D);
}

// CS critical point: on the spinodal T(eta) is proportional to
// eta (1 - eta)^4 / (1 + 4 eta + 4 eta^2 - 4 eta^3 + eta^4); bisection on the
// zero of its logarithmic derivative.
void critical_point_cs(double a, double b, double R, double* rho_c, double* T_c) {
    auto q = [](double e) { return 1.0 + e * (4.0 + e * (4.0 + e * (-4.0 + e))); };
    auto dlog = [&](double e) {
        const double dq = 4.0 + e * (8.0 + e * (-12.0 + 4.0 * e));
        return 1.0 / e - 4.0 / (1.0 - e) - dq / q(e);
    };
    double lo = 1e-6, hi = 1.0 - 1e-6;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (dlog(mid) > 0.0) lo = mid; else hi = mid;
    }
    const double e = 0.5 * (lo + hi), o = 1.0 - e;
    *rho_c = 4.0 * e / b;
    *T_c = 2.0 * a * (*rho_c) * o * o * o * o / (R * q(e));
}

// the critical point of the EOS that the flags select
void critical_of(const lbm_params& p, double* rho_c, double* T_c) {
    if (p.flags & LBM_EOS_CS) critical_point_cs(p.a, p.b, p.R, rho_c, T_c);
    else critical_point(p.a, p.b, p.R, rho_c, T_c);
}

Eos eos_of(const lbm_params& p, double Tc) {
    Eos E{p.a, p.b, p.R, kappa_of(p.omega), Tc};
    E.cs = (p.flags & LBM_EOS_CS) != 0;
    return E;
}

// Open ends (LBM_OPEN_X): the boundary EOS pressures are taken at the inlet
// temperature; p0 = P_EOS(rho_v, T_in).  The inlet density is a root on the
// vapour branch, below the vapour spinodal (first zero of dP/drho; the
// packing limit when the isotherm has none).
double inlet_temperature(const lbm_params& p) { return p.T_in > 0.0 ? p.T_in : p.T_0; }
double inlet_p0(const lbm_params& p) {
    double Tc = p.T_c, rc;
    if (!(Tc > 0.0)) critical_of(p, &rc, &Tc);
    return eos_of(p, Tc).P(p.rho_v, inlet_temperature(p));
}
bool inlet_bracket(const lbm_params& p, double* rho_sp, double* p_max, void*) {
    double Tc = p.T_c, rc;
    if (!(Tc > 0.0)) critical_of(p, &rc, &Tc);
    const Eos E = eos_of(p, Tc);
    const double T = inlet_temperature(p), rmax = E.rmax();
    if (!(T > 0.0)) return false;
    double hi = rmax * (1.0 - 1e-9);
    const int n = 8192;
    double prev = rmax * 1e-9;
    for (int i = 1; i < n; ++i) {
        const double r = rmax * i / n;
        if (E.dPdr(r, T) <= 0.0) {
            double lo = prev, h = r;
            for (int it = 0; it < 100; ++it) {
                const double mid = 0.5 * (lo + h);
                if (E.dPdr(mid, T) > 0.0) lo = mid; else h = mid;
            }
            hi = lo;
            break;
        }
        prev = r;
    }
    if (rho_sp) *rho_sp = hi;
    if (p_max) *p_max = E.P(hi, T);
    return true;
}

template <class F>
double bisect(F f, double lo, double hi) {
    const double flo = f(lo);
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi), fm = f(mid);
        if ((fm > 0.0) == (flo > 0.0)) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

// Coexistence at T: equal pressure and equal chemical potential.  For a trial
// pressure p between the spinodal pressures the vapour and liquid roots of
// P = p are bracketed; mu(liquid) - mu(vapour) changes sign at p_sat.
bool coexistence(const Eos& E, double T, double* rg, double* rl, double* ps) {
    const double rmax = E.rmax();
    const int n = 4000;
    double s1 = -1.0, s2 = -1.0;
    double prev = E.dPdr(rmax * 1e-6, T);
    for (int i = 1; i < n; ++i) {
        const double r = rmax * i / n;
        const double cur = E.dPdr(r, T);
        if (prev > 0.0 && cur <= 0.0 && s1 < 0.0)
            s1 = bisect([&](double x) { return E.dPdr(x, T); }, rmax * (i - 1) / n, r);
        if (prev <= 0.0 && cur > 0.0 && s1 > 0.0)
            s2 = bisect([&](double x) { return E.dPdr(x, T); }, rmax * (i - 1) / n, r);
        prev = cur;
    }
    if (s1 < 0.0 || s2 < 0.0) return false;
    const double pmax = E.P(s1, T), pmin = std::max(E.P(s2, T), 1e-300);
    double g = 0, l = 0;
    auto dmu = [&](double p) {
        g = bisect([&](double x) { return E.P(x, T) - p; }, 1e-300, s1);
        l = bisect([&](double x) { return E.P(x, T) - p; }, s2, rmax * (1.0 - 1e-15));
        return E.mu(l, T) - E.mu(g, T);
    };
    const double p = bisect(dmu, pmin, pmax);
    dmu(p);
    *rg = g;
    *rl = l;
    *ps = p;
    return true;
}

}  // namespace

namespace lbmhost {

bool make_layout(const lbm_params& p, Layout* L) {
    // a grid whose step buffers fit the 32-bit offsets is far below these
    // bounds; larger ones are refused before any index arithmetic
    if (p.Nx < 1 || p.Ny < 1 || p.Nx > (1 << 28) || p.Ny > (1 << 28)) return false;
    const bool per = (p.flags & LBM_PERIODIC_Y) != 0;
    L->pitch = (p.Nx + 63) / 64 * 64;
    L->rows = per ? p.Ny : p.Ny - 2;
    L->plane = (size_t)L->pitch * L->rows + kPlaneSkew;
    L->esz = p.precision == LBM_FP64 ? 8 : 4;

    const size_t cells = (size_t)p.Nx * p.Ny;
    size_t o = 0;
    for (int b = 0; b < 2; ++b) {
        L->off_f[b] = o;
        o = align_up(o + 9 * L->plane * L->esz);
    }
    for (int b = 0; b < 2; ++b) {
        L->off_lo[b] = o;
        if (p.precision == LBM_FP32_DEV_MASSEXACT) o = align_up(o + L->plane * 4);
    }
    for (int b = 0; b < 2; ++b) {
        L->off_T[b] = o;
        o = align_up(o + L->plane * L->esz);
    }
    // the step reaches its buffers by 32-bit byte offsets from the base
    if (o >= ((size_t)1 << 32) - kAlign) return false;
    L->off_mom = o;
    o = align_up(o + 4 * cells * sizeof(double));
    L->off_scr = o;
    o = align_up(o + 3 * cells * sizeof(double));
    L->off_part = o;
    o = align_up(o + lbmk::kReduceBlocks * 5 * sizeof(double));
    L->off_out = o;
    o = align_up(o + 8 * sizeof(double));
    L->off_stat = o;
    o = align_up(o + kStatWords * sizeof(unsigned long long));
    L->total = o;
    return true;
}

lbm_status validate(const lbm_params& p) {
    const bool per = (p.flags & LBM_PERIODIC_Y) != 0;
    if (p.Nx < 3) return fail(LBM_EINVAL, "Nx = %d < 3", p.Nx);
    if (p.Ny < (per ? 3 : 4)) return fail(LBM_EINVAL, "Ny = %d too small", p.Ny);
    if (p.precision < LBM_FP32_DEV || p.precision > LBM_FP32_DEV_MASSEXACT)
        return fail(LBM_EINVAL, "unknown precision %d", p.precision);
    if (p.flags & ~511u) return fail(LBM_EINVAL, "unknown flags 0x%x", p.flags);
    if (p.flags & LBM_TOP_MIXED) {
        if (p.flags & (LBM_PERIODIC_Y | LBM_OPEN_X))
            return fail(LBM_EINVAL, "LBM_TOP_MIXED needs plates and periodic x");
        if (p.T_w_end > 0.0) return fail(LBM_EINVAL, "LBM_TOP_MIXED excludes T_w_end > 0");
        if (!(0 <= p.cold_x0 && p.cold_x0 <= p.cold_x1 && p.cold_x1 <= p.Nx))
            return fail(LBM_EINVAL, "LBM_TOP_MIXED needs 0 <= cold_x0 <= cold_x1 <= Nx");
    }
    if ((p.flags & LBM_PHASE_PROPS) && !(p.lambda_l >= 0.0 && p.C_v_l > 0.0))
        return fail(LBM_EINVAL, "LBM_PHASE_PROPS needs lambda_l >= 0 and C_v_l > 0");
    if (p.flags & LBM_OPEN_X) {
        if (p.Nx < 4) return fail(LBM_EINVAL, "LBM_OPEN_X needs Nx >= 4");
        double pmax;
        if (!inlet_bracket(p, nullptr, &pmax, nullptr))
            return fail(LBM_EINVAL, "LBM_OPEN_X: no vapour state at the inlet temperature");
        const double p0 = inlet_p0(p);
        if (!(p0 * (1.0 + std::fabs(p.p_amp)) < pmax) || !(p0 * (1.0 - std::fabs(p.p_amp)) > 0.0))
            return fail(LBM_EINVAL, "LBM_OPEN_X: inlet pressure range leaves the vapour branch");
    }
    if (!(p.alpha_max == 0.0 || (p.alpha_max > 0.0 && p.alpha_max <= 0.522)))
        return fail(LBM_EINVAL, "alpha_max must be 0 (off) or in (0, 0.522]");
    if (p.T_out != 0.0 && !((p.flags & LBM_OPEN_X) && p.T_out > 0.0))
        return fail(LBM_EINVAL, "T_out must be 0, or positive with LBM_OPEN_X");
    if ((p.flags & LBM_FRAME_RHO) && !(p.rho_frame > 0.0))
        return fail(LBM_EINVAL, "LBM_FRAME_RHO needs rho_frame > 0");
    if (p.G == 0.0) return fail(LBM_EINVAL, "G must be nonzero");
    const double rates[5] = {p.s_rho, p.s_e, p.s_zeta, p.s_j, p.s_q};
    for (double s : rates)
        if (!(s > 0.0 && s < 2.0)) return fail(LBM_EINVAL, "relaxation rate %g outside (0, 2)", s);
    if (p.s_e != p.s_zeta) return fail(LBM_EINVAL, "Eq. 3 requires s_e == s_zeta");
    if (!(p.tau_g > 0.5 && p.tau_l > 0.5)) return fail(LBM_EINVAL, "tau must exceed 1/2");
    if (!(p.a > 0.0 && p.b > 0.0 && p.R > 0.0 && p.T_c > 0.0))
        return fail(LBM_EINVAL, "EOS constants must be positive");
    if (!(p.T_0 > 0.0 && p.T_w > 0.0)) return fail(LBM_EINVAL, "temperatures must be positive");
    if (!(p.C_v > 0.0) || p.lambda < 0.0) return fail(LBM_EINVAL, "C_v > 0, lambda >= 0 needed");
    if (!(p.rho_ref > 0.0)) return fail(LBM_EINVAL, "rho_ref must be positive");
    Layout L;
    if (!make_layout(p, &L)) return fail(LBM_EINVAL, "grid too large: the step buffers must stay below 4 GiB");
    return LBM_OK;
}

lbm_status check_initial(const lbm_params& p, const double* rho0) {
    const bool per = (p.flags & LBM_PERIODIC_Y) != 0;
    const Eos E = eos_of(p, p.T_c);
    const double T_in = (p.flags & LBM_OPEN_X) ? inlet_temperature(p) : p.T_0;
    for (int y = per ? 0 : 1; y < (per ? p.Ny : p.Ny - 1); ++y)
        for (int x = 0; x < p.Nx; ++x) {
            const double r = rho0 ? rho0[(size_t)y * p.Nx + x] : p.rho_v;
            if (!(r > 0.0 && r < E.rmax()))
                return fail(LBM_EINVAL, "initial density %g at (%d, %d) outside the EOS range",
                            r, x, y);
            // the initial temperature of the node (as the start state sets it)
            const bool frame = x == 0 || x == p.Nx - 1 || (per && (y == 0 || y == p.Ny - 1));
            double T = p.T_0;
            if ((p.flags & LBM_OPEN_X) && x == 0) T = T_in;
            else if ((p.flags & LBM_OPEN_X) && x == p.Nx - 1 && p.T_out > 0.0) T = p.T_out;
            else if ((p.flags & LBM_FRAME_T) && frame) T = p.T_w;
            const double rr = ((p.flags & LBM_FRAME_RHO) && frame) ? p.rho_frame : r;
            const double arg = 2.0 * (E.P(rr, T) - rr / 3.0) / p.G;
            if (!(arg >= 0.0))
                return fail(LBM_EINVAL,
                            "initial density %g at (%d, %d) leaves Eq. 10 without a real psi "
                            "(2 (P - rho/3) / G = %g at T = %g)", rr, x, y, arg, T);
        }
    return LBM_OK;
}

}  // namespace lbmhost

using lbmhost::align_up;
using lbmhost::kAlign;
using lbmhost::make_layout;
using lbmhost::validate;

struct lbm_sim {
    lbm_params p;
    Grid g;
    Phys k;
    Layout L;
    int dev = 0;
    char* base = nullptr;
    bool owns_mem = false;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    int64_t n = 0;
    int fcur = 0, tcur = 0;
    int seg_rows = 0;

    template <class S>
    S* f(int b) const { return reinterpret_cast<S*>(base + L.off_f[b]); }
    template <class S>
    S* T(int b) const { return reinterpret_cast<S*>(base + L.off_T[b]); }
    float* lo(int b) const {
        return p.precision == LBM_FP32_DEV_MASSEXACT ? reinterpret_cast<float*>(base + L.off_lo[b])
                                                     : nullptr;
    }
    double* mom(int q) const {
        return reinterpret_cast<double*>(base + L.off_mom) + (size_t)q * p.Nx * p.Ny;
    }
    double* scr() const { return reinterpret_cast<double*>(base + L.off_scr); }
    double* part() const { return reinterpret_cast<double*>(base + L.off_part); }
    double* out() const { return reinterpret_cast<double*>(base + L.off_out); }
    unsigned long long* stat() const {
        return reinterpret_cast<unsigned long long*>(base + L.off_stat);
    }
};

namespace lbmhost {

// default launch shape: enough waves to give each of the 1024 SIMDs about two
// (the register budget of the fused kernel allows two resident per SIMD), but
// segments of at least 16 rows so the 10 recomputed halo rows stay a minority.
int default_seg_rows(const lbm_params& p, int rows, int min_rows) {
    const int strips = (p.Nx + lbmk::kOwned - 1) / lbmk::kOwned;
    // one resident round: 256 CUs x 4 SIMDs x 3 waves for the FP32 deviation
    // build, 2 waves for the FP64 and mass-exact builds
    const int want_units = p.precision == LBM_FP32_DEV ? 3072 : 2048;
    int segs = std::max(1, (want_units + strips - 1) / strips);
    int sr = (rows + segs - 1) / segs;
    sr = std::max(sr, min_rows);
    sr = sr + (6 - (sr + 10) % 6) % 6;  // seg + 10 a multiple of the 6-row unroll
    return std::min(sr, rows);
}

void fill_grid(const lbm_params& p, const Layout& L, int seg_rows, Grid& g) {
    g.Nx = p.Nx;
    g.Ny = p.Ny;
    g.pitch = L.pitch;
    g.rows = L.rows;
    g.periodic_y = (p.flags & LBM_PERIODIC_Y) ? 1 : 0;
    g.frame_t = (p.flags & LBM_FRAME_T) ? 1 : 0;
    g.frame_rho = (p.flags & LBM_FRAME_RHO) ? 1 : 0;
    g.open_x = (p.flags & LBM_OPEN_X) ? 1 : 0;
    g.y_first = g.periodic_y ? 0 : 1;
    g.plane = (unsigned)L.plane;
    g.n_strips = (p.Nx + lbmk::kOwned - 1) / lbmk::kOwned;
    g.seg_rows = std::max(1, std::min(seg_rows, g.rows));
    g.n_segs = (g.rows + g.seg_rows - 1) / g.seg_rows;
    g.n_units = g.n_strips * g.n_segs;
    const int nb = (g.n_units + lbmk::kWavesPerBlock - 1) / lbmk::kWavesPerBlock;
    g.n_blocks_pad = (nb + 7) / 8 * 8;
}

void fill_phys(const lbm_params& p, Phys& k) {
    std::memset(&k, 0, sizeof(k));
    const double kap = kappa_of(p.omega);
    k.rho_ref = p.rho_ref;
    k.T_ref = p.T_0;
    k.dT_wall = p.T_w - p.T_0;
    k.a = p.a;
    k.b = p.b;
    k.R = p.R;
    k.kappa = kap;
    k.inv_Tc = 1.0 / p.T_c;
    k.inv_G = 1.0 / p.G;
    k.negG = -p.G;
    k.psi_wall_eff = p.psi_w * p.G_w / p.G;
    k.Gw_psiw = p.G_w * p.psi_w;
    k.c_e = 12.0 * p.theta / (1.0 / p.s_e - 0.5);
    k.c_z = 12.0 * p.theta / (1.0 / p.s_zeta - 0.5);
    k.s_rho = p.s_rho;
    k.s_e = p.s_e;
    k.s_z = p.s_zeta;
    k.s_j = p.s_j;
    k.s_q = p.s_q;
    k.tau_g = p.tau_g;
    k.dtau = p.tau_l - p.tau_g;
    k.rho_g = p.rho_g;
    k.inv_drho = (p.rho_l != p.rho_g) ? 1.0 / (p.rho_l - p.rho_g) : 0.0;
    k.inv_Cv = 1.0 / p.C_v;
    k.lambda = p.lambda;
    k.g_osc = p.g_osc;
    k.period = p.period;
    k.g_x = p.g_x;
    k.g_y = p.g_y;
    k.rho_v = p.rho_v;
    k.rho_frame = p.rho_frame;
    if (p.flags & LBM_OPEN_X) {
        k.T_in_eos = p.T_in > 0.0 ? p.T_in : p.T_0;
        k.p0 = inlet_p0(p);
        inlet_bracket(p, &k.rho_sp, nullptr, nullptr);
        k.p_amp = p.p_amp;
        k.p_period = p.p_period;
    }
    k.dT_in = (p.T_in > 0.0 ? p.T_in : p.T_0) - p.T_0;
    k.hold_out = (p.flags & LBM_OPEN_X) && p.T_out > 0.0 ? 1 : 0;
    k.dT_out = k.hold_out ? p.T_out - p.T_0 : 0.0;
    k.alpha_max = p.alpha_max > 0.0 ? p.alpha_max : 0.0;
    k.wall_ramp = p.T_w_end > 0.0 ? 1 : 0;
    k.lam_l = p.lambda_l;
    k.cv_l = p.C_v_l;
    k.dT_w_end = (p.T_w_end > 0.0 ? p.T_w_end : p.T_w) - p.T_0;
    k.dT_w_bot = (p.flags & LBM_TOP_MIXED) ? (p.T_w_bottom > 0.0 ? p.T_w_bottom : p.T_0) - p.T_0
                                           : k.dT_wall;
    k.cold_x0 = p.cold_x0;
    k.cold_x1 = p.cold_x1;
    k.rkA = p.R;
    k.rkB1 = p.a * kap * (1.0 + kap) / std::sqrt(p.T_c);
    k.rkB2 = p.a * kap * kap / p.T_c;
    if (p.flags & LBM_EOS_CS) {  // no temperature-dependent attraction
        k.kappa = 0.0;
        k.rkB1 = k.rkB2 = 0.0;
    }
    k.flags = p.flags;
    auto fillr = [&](auto& r) {
        using T = std::remove_reference_t<decltype(r.b)>;
        r.s_rho = (T)k.s_rho;
        r.s_e = (T)k.s_e;
        r.s_z = (T)k.s_z;
        r.s_j = (T)k.s_j;
        r.s_q = (T)k.s_q;
        r.c_e = (T)k.c_e;
        r.c_z = (T)k.c_z;
        r.b = (T)k.b;
        r.rkA = (T)k.rkA;
        r.rkB1 = (T)k.rkB1;
        r.rkB2 = (T)k.rkB2;
        r.inv_Cv = (T)k.inv_Cv;
        r.lambda = (T)k.lambda;
        r.T_ref = (T)k.T_ref;
        r.dT_wall = (T)k.dT_wall;
        r.rho_ref = (T)k.rho_ref;
        r.rho_v = (T)k.rho_v;
        r.g_x = (T)k.g_x;
        r.g_y = (T)k.g_y;
        r.rho_g = (T)k.rho_g;
        r.inv_drho = (T)k.inv_drho;
        r.tau_g = (T)k.tau_g;
        r.dtau = (T)k.dtau;
    };
    fillr(k.rf);
    fillr(k.rd);
}

}  // namespace lbmhost

namespace {

using lbmhost::default_seg_rows;

void set_grid(lbm_sim* s, int seg_rows) {
    lbmhost::fill_grid(s->p, s->L, seg_rows, s->g);
    s->seg_rows = s->g.seg_rows;
}

void set_phys(lbm_sim* s) { lbmhost::fill_phys(s->p, s->k); }

hipError_t enqueue_step(lbm_sim* s) {
    const int fa = s->fcur, fb = 1 - s->fcur;
    const int ta = s->tcur, tb = (s->p.flags & LBM_FREEZE_T) ? s->tcur : 1 - s->tcur;
    hipError_t e;
    const unsigned span = (unsigned)(s->L.off_T[1] + s->L.plane * s->L.esz);
    const auto off = [](size_t o) { return (unsigned)o; };
    if (s->p.precision == LBM_FP64) {
        lbmk::Bufs<double> b{s->base, span, off(s->L.off_f[fa]), off(s->L.off_f[fb]), 0u, 0u,
                             off(s->L.off_T[ta]), off(s->L.off_T[tb]), s->stat()};
        e = lbmk::launch_step_f64(s->g, s->k, b, s->n, s->stream);
    } else {
        lbmk::Bufs<float> b{s->base, span, off(s->L.off_f[fa]), off(s->L.off_f[fb]),
                            off(s->L.off_lo[fa]), off(s->L.off_lo[fb]),
                            off(s->L.off_T[ta]), off(s->L.off_T[tb]), s->stat()};
        e = lbmk::launch_step_f32(s->g, s->k, b, s->p.precision == LBM_FP32_DEV_MASSEXACT, s->n,
                                  s->stream);
    }
    if (e != hipSuccess) return e;
    s->fcur = fb;
    s->tcur = tb;
    s->n += 1;
    return hipSuccess;
}

// The read-out's count of non-finite nodes restarts at every read-out.
hipError_t enqueue_moments(lbm_sim* s) {
    unsigned long long* nb = s->stat() + lbmhost::kStatReadout;
    hipError_t e = hipMemsetAsync(nb, 0, sizeof(*nb), s->stream);
    if (e != hipSuccess) return e;
    if (s->p.precision == LBM_FP64)
        return lbmk::launch_moments_f64(s->g, s->k, s->f<double>(s->fcur), s->T<double>(s->tcur),
                                        s->scr(), s->mom(0), s->mom(1), s->mom(2), s->mom(3),
                                        s->n, nb, s->stream);
    return lbmk::launch_moments_f32(s->g, s->k, s->f<float>(s->fcur), s->lo(s->fcur),
                                    s->T<float>(s->tcur), s->scr(), s->mom(0), s->mom(1),
                                    s->mom(2), s->mom(3), s->n, nb, s->stream);
}

// Host copy of the health counters, enqueued on the stream (the caller
// synchronises).
hipError_t enqueue_stat_copy(lbm_sim* s, unsigned long long* host) {
    return hipMemcpyAsync(host, s->stat(), lbmhost::kStatWords * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, s->stream);
}

// LBM_EUNSTABLE (with the counts in the message) when any step read a
// non-finite state or the read-out found one; LBM_OK otherwise.
lbm_status health_status(const lbm_sim* s, const unsigned long long* st, bool readout) {
    const unsigned long long bad = st[lbmhost::kStatNonfinite],
                             now = readout ? st[lbmhost::kStatReadout] : 0ull;
    if (bad || now)
        return fail(LBM_EUNSTABLE,
                    "non-finite state: %llu node readings by the steps up to n = %lld, "
                    "%llu nodes at the read-out", bad, (long long)s->n, now);
    return LBM_OK;
}

size_t state_payload(const lbm_sim* s) {
    size_t b = 9 * s->L.plane * s->L.esz + s->L.plane * s->L.esz;
    if (s->p.precision == LBM_FP32_DEV_MASSEXACT) b += s->L.plane * 4;
    return b;
}

struct CkptHeader {
    char magic[8];
    int64_t n;
    lbm_params p;
};

}  // namespace

extern "C" {

void lbm_params_default(lbm_params* p) {
    std::memset(p, 0, sizeof(*p));
    p->Nx = 128;
    p->Ny = 32;
    p->a = 3.0 / 49.0;
    p->b = 2.0 / 21.0;
    p->R = 1.0;
    p->omega = 0.344;
    p->T_c = 0.0;
    p->G = -1.0;
    p->theta = 0.104;
    p->G_w = 0.0;
    p->psi_w = 0.0;
    p->s_rho = 1.0;
    p->s_e = 0.8;
    p->s_zeta = 0.8;
    p->s_j = 1.0;
    p->s_q = 1.1;
    p->tau_g = 1.0;
    p->tau_l = 1.0;
    p->C_v = 5.0;
    p->lambda = 0.25;
    p->g_osc = 1e-6;
    p->period = 2000.0;
    p->rho_v = -1.0;
    p->precision = LBM_FP32_DEV;
    p->flags = 0;
}

lbm_status lbm_eos_critical(double a, double b, double R, double* rho_c, double* T_c) {
    if (!(a > 0 && b > 0 && R > 0) || !rho_c || !T_c)
        return fail(LBM_EINVAL, "EOS constants must be positive");
    critical_point(a, b, R, rho_c, T_c);
    return LBM_OK;
}

lbm_status lbm_eos_critical_cs(double a, double b, double R, double* rho_c, double* T_c) {
    if (!(a > 0 && b > 0 && R > 0) || !rho_c || !T_c)
        return fail(LBM_EINVAL, "EOS constants must be positive");
    critical_point_cs(a, b, R, rho_c, T_c);
    return LBM_OK;
}

lbm_status lbm_eos_coexistence(const lbm_params* p, double T, double* rho_g, double* rho_l,
                               double* p_sat) {
    if (!p || !rho_g || !rho_l || !p_sat) return fail(LBM_EINVAL, "null argument");
    double Tc = p->T_c, rc;
    if (!(Tc > 0.0)) critical_of(*p, &rc, &Tc);
    if (!(T > 0.0 && T < Tc)) return fail(LBM_EINVAL, "T = %g is not below Tc = %g", T, Tc);
    const Eos E = eos_of(*p, Tc);
    if (!coexistence(E, T, rho_g, rho_l, p_sat))
        return fail(LBM_EINVAL, "no coexistence found at T = %g", T);
    return LBM_OK;
}

lbm_status lbm_eos_pressure(const lbm_params* p, double rho, double T, double* P, double* psi) {
    if (!p) return fail(LBM_EINVAL, "null params");
    if (p->G == 0.0) return fail(LBM_EINVAL, "G must be nonzero");
    double Tc = p->T_c, rc;
    if (!(Tc > 0.0)) critical_of(*p, &rc, &Tc);
    const Eos E = eos_of(*p, Tc);
    if (!(rho > 0.0 && rho < E.rmax() && T > 0.0)) return fail(LBM_EINVAL, "rho or T out of range");
    const double pe = E.P(rho, T);
    const double arg = 2.0 * (pe - rho / 3.0) / p->G;
    if (P) *P = pe;
    if (psi) *psi = arg > 0.0 ? std::sqrt(arg) : 0.0;
    return LBM_OK;
}

lbm_status lbm_eos_latent_heat(const lbm_params* p, double T, double* h_fg) {
    if (!p || !h_fg) return fail(LBM_EINVAL, "null argument");
    double rg, rl, ps;
    const lbm_status st = lbm_eos_coexistence(p, T, &rg, &rl, &ps);
    if (st != LBM_OK) return st;
    if (p->flags & LBM_EOS_CS) {  // T-independent attraction a rho^2: du = -a drho
        *h_fg = p->a * (rl - rg) + ps * (1.0 / rg - 1.0 / rl);
        return LBM_OK;
    }
    double Tc = p->T_c, rc;
    if (!(Tc > 0.0)) critical_point(p->a, p->b, p->R, &rc, &Tc);
    const double k = kappa_of(p->omega), b = p->b, s2 = std::sqrt(2.0);
    const double sq = std::sqrt(T / Tc), s = 1.0 + k * (1.0 - sq);
    // a phi - T a phi' with phi = s^2, T phi' = -k s sqrt(T/Tc)
    const double attr = p->a * (s * s + k * s * sq);
    auto L = [&](double r) {
        return std::log((1.0 + (1.0 + s2) * b * r) / (1.0 + (1.0 - s2) * b * r));
    };
    *h_fg = attr / (2.0 * s2 * b) * (L(rl) - L(rg)) + ps * (1.0 / rg - 1.0 / rl);
    return LBM_OK;
}

lbm_status lbm_eos_jacob(const lbm_params* p, double T_sat, double T_w, double* Ja) {
    if (!p || !Ja) return fail(LBM_EINVAL, "null argument");
    double h;
    const lbm_status st = lbm_eos_latent_heat(p, T_sat, &h);
    if (st != LBM_OK) return st;
    *Ja = p->C_v * (T_sat - T_w) / h;
    return LBM_OK;
}

lbm_status lbm_params_resolve(lbm_params* p) {
    if (!p) return fail(LBM_EINVAL, "null params");
    if (!(p->a > 0 && p->b > 0 && p->R > 0)) return fail(LBM_EINVAL, "EOS constants must be positive");
    if (!(p->T_c > 0.0)) {
        double rc;
        critical_of(*p, &rc, &p->T_c);
    }
    if (!(p->T_0 > 0.0)) p->T_0 = 0.86 * p->T_c;
    if (!(p->T_w > 0.0)) p->T_w = 0.80 * p->T_c;
    double g = 0.0;
    if (!(p->rho_g > 0.0) || !(p->rho_l > 0.0) || p->rho_v < 0.0 || !(p->rho_ref > 0.0)) {
        double l, ps;
        lbm_status st = lbm_eos_coexistence(p, p->T_0, &g, &l, &ps);
        if (st != LBM_OK) return st;
        if (!(p->rho_g > 0.0)) p->rho_g = g;
        if (!(p->rho_l > 0.0)) p->rho_l = l;
        if (p->rho_v < 0.0) p->rho_v = g;
    }
    if (!(p->rho_ref > 0.0)) p->rho_ref = p->rho_v > 0.0 ? p->rho_v : g;
    return LBM_OK;
}

size_t lbm_workspace_bytes(const lbm_params* pin) {
    if (!pin) return 0;
    lbm_params p = *pin;
    if (lbm_params_resolve(&p) != LBM_OK || validate(p) != LBM_OK) return 0;
    Layout L;
    make_layout(p, &L);
    return L.total;
}

lbm_status lbm_create(const lbm_params* pin, const double* rho0, void* workspace,
                      size_t ws_bytes, void* stream, lbm_sim** out) {
    if (!out) return fail(LBM_EINVAL, "null output handle");
    *out = nullptr;
    if (!pin) return fail(LBM_EINVAL, "null params");
    lbm_params p = *pin;
    lbm_status st = lbm_params_resolve(&p);
    if (st != LBM_OK) return st;
    st = validate(p);
    if (st != LBM_OK) return st;
    const size_t cells = (size_t)p.Nx * p.Ny;
    st = lbmhost::check_initial(p, rho0);
    if (st != LBM_OK) return st;
    std::vector<double> r0(cells, p.rho_v);
    if (rho0) std::copy(rho0, rho0 + cells, r0.begin());

    lbm_sim* s = new (std::nothrow) lbm_sim();
    if (!s) return fail(LBM_ENOMEM, "host allocation failed");
    s->p = p;
    make_layout(p, &s->L);
    hipError_t e = hipGetDevice(&s->dev);
    if (e != hipSuccess) {
        delete s;
        return fail(LBM_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    }
    if (workspace) {
        if (ws_bytes < s->L.total || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0) {
            delete s;
            return fail(LBM_EINVAL, "workspace needs %zu bytes aligned to %d", s->L.total, kAlign);
        }
        s->base = static_cast<char*>(workspace);
    } else {
        e = hipMalloc(reinterpret_cast<void**>(&s->base), s->L.total);
        if (e != hipSuccess) {
            delete s;
            return fail(LBM_ENOMEM, "hipMalloc(%zu): %s", s->L.total, hipGetErrorString(e));
        }
        s->owns_mem = true;
    }
    if (stream) {
        s->stream = static_cast<hipStream_t>(stream);
    } else {
        e = hipStreamCreate(&s->stream);
        if (e != hipSuccess) {
            lbm_destroy(s);
            return fail(LBM_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        }
        s->owns_stream = true;
    }
    set_phys(s);
    set_grid(s, default_seg_rows(p, s->L.rows));
    // zero everything (pitch padding stays zero), upload rho0, start state
    e = hipMemsetAsync(s->base, 0, s->L.total, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->mom(0), r0.data(), cells * sizeof(double), hipMemcpyHostToDevice,
                           s->stream);
    if (e == hipSuccess) {
        if (p.precision == LBM_FP64)
            e = lbmk::launch_init_f64(s->g, s->k, s->mom(0), s->f<double>(0), s->T<double>(0),
                                      s->stream);
        else
            e = lbmk::launch_init_f32(s->g, s->k, s->mom(0), s->f<float>(0), s->lo(0),
                                      s->T<float>(0), s->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);  // r0 must outlive the copy
    if (e != hipSuccess) {
        lbm_destroy(s);
        return fail(LBM_EDEVICE, "initialisation: %s", hipGetErrorString(e));
    }
    *out = s;
    return LBM_OK;
}

lbm_status lbm_step(lbm_sim* s, int64_t n) {
    if (!s) return fail(LBM_EINVAL, "null sim");
    if (n < 0) return fail(LBM_EINVAL, "negative step count");
    HIPCHK(hipSetDevice(s->dev));
    for (int64_t i = 0; i < n; ++i) HIPCHK(enqueue_step(s));
    return LBM_OK;
}

lbm_status lbm_synchronize(lbm_sim* s) {
    if (!s) return fail(LBM_EINVAL, "null sim");
    HIPCHK(hipSetDevice(s->dev));
    unsigned long long st[lbmhost::kStatWords];
    HIPCHK(enqueue_stat_copy(s, st));
    HIPCHK(hipStreamSynchronize(s->stream));
    return health_status(s, st, false);
}

lbm_status lbm_moments(lbm_sim* s, double* rho, double* ux, double* uy, double* T) {
    if (!s) return fail(LBM_EINVAL, "null sim");
    HIPCHK(hipSetDevice(s->dev));
    HIPCHK(enqueue_moments(s));
    double* outs[4] = {rho, ux, uy, T};
    const size_t bytes = (size_t)s->p.Nx * s->p.Ny * sizeof(double);
    for (int q = 0; q < 4; ++q)
        if (outs[q])
            HIPCHK(hipMemcpyAsync(outs[q], s->mom(q), bytes, hipMemcpyDeviceToHost, s->stream));
    unsigned long long st[lbmhost::kStatWords];
    HIPCHK(enqueue_stat_copy(s, st));
    HIPCHK(hipStreamSynchronize(s->stream));
    return health_status(s, st, true);
}

lbm_status lbm_reduce(lbm_sim* s, double out[5]) {
    if (!s || !out) return fail(LBM_EINVAL, "null argument");
    HIPCHK(hipSetDevice(s->dev));
    HIPCHK(enqueue_moments(s));
    HIPCHK(lbmk::launch_reduce(s->mom(0), s->mom(1), s->mom(2), s->mom(3), s->p.Nx * s->p.Ny,
                               s->p.C_v, s->part(), s->out(), s->stream));
    HIPCHK(hipMemcpyAsync(out, s->out(), 5 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    unsigned long long st[lbmhost::kStatWords];
    HIPCHK(enqueue_stat_copy(s, st));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (out[4] > 0.0) return fail(LBM_EUNSTABLE, "%g non-finite nodes at n = %lld", out[4],
                                  (long long)s->n);
    return health_status(s, st, true);
}

lbm_status lbm_reduce_noalloc(lbm_sim* s, double* out_dev) {
    if (!s || !out_dev) return fail(LBM_EINVAL, "null argument");
    if ((reinterpret_cast<uintptr_t>(out_dev) & 7u) != 0)
        return fail(LBM_EINVAL, "out_dev must be 8-byte aligned");
    HIPCHK(hipSetDevice(s->dev));
    if (s->p.precision == LBM_FP64)
        HIPCHK(lbmk::launch_reduce_state_f64(s->g, s->k, s->f<double>(s->fcur),
                                             s->T<double>(s->tcur), s->p.C_v, s->n, out_dev,
                                             s->stream));
    else
        HIPCHK(lbmk::launch_reduce_state_f32(s->g, s->k, s->f<float>(s->fcur), s->lo(s->fcur),
                                             s->T<float>(s->tcur), s->p.C_v, s->n, out_dev,
                                             s->stream));
    return LBM_OK;
}

lbm_status lbm_health(lbm_sim* s, int64_t* nonfinite, int64_t* psi_clamps) {
    if (!s) return fail(LBM_EINVAL, "null sim");
    HIPCHK(hipSetDevice(s->dev));
    unsigned long long st[lbmhost::kStatWords];
    HIPCHK(enqueue_stat_copy(s, st));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (nonfinite) *nonfinite = (int64_t)st[lbmhost::kStatNonfinite];
    if (psi_clamps) *psi_clamps = (int64_t)st[lbmhost::kStatClamps];
    return LBM_OK;
}

lbm_status lbm_destroy(lbm_sim* s) {
    if (!s) return LBM_OK;
    (void)hipSetDevice(s->dev);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->owns_mem && s->base) (void)hipFree(s->base);
    if (s->owns_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return LBM_OK;
}

int64_t lbm_time(const lbm_sim* s) { return s ? s->n : -1; }

lbm_status lbm_get_params(const lbm_sim* s, lbm_params* out) {
    if (!s || !out) return fail(LBM_EINVAL, "null argument");
    *out = s->p;
    return LBM_OK;
}

const char* lbm_last_error(void) { return g_err; }

// Checkpoint magic; the number changes whenever the header (which holds
// lbm_params) changes layout.
constexpr char kCkptMagic[9] = "LBMCKPT4";

size_t lbm_state_bytes(const lbm_sim* s) {
    return s ? sizeof(CkptHeader) + state_payload(s) : 0;
}

lbm_status lbm_save(lbm_sim* s, void* host, size_t bytes) {
    if (!s || !host) return fail(LBM_EINVAL, "null argument");
    if (bytes < lbm_state_bytes(s)) return fail(LBM_EINVAL, "buffer too small");
    HIPCHK(hipSetDevice(s->dev));
    CkptHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, kCkptMagic, 8);
    h.n = s->n;
    h.p = s->p;
    char* dst = static_cast<char*>(host);
    std::memcpy(dst, &h, sizeof(h));
    dst += sizeof(h);
    const size_t fb = 9 * s->L.plane * s->L.esz, tb = s->L.plane * s->L.esz;
    HIPCHK(hipMemcpyAsync(dst, s->base + s->L.off_f[s->fcur], fb, hipMemcpyDeviceToHost, s->stream));
    dst += fb;
    HIPCHK(hipMemcpyAsync(dst, s->base + s->L.off_T[s->tcur], tb, hipMemcpyDeviceToHost, s->stream));
    dst += tb;
    if (s->p.precision == LBM_FP32_DEV_MASSEXACT)
        HIPCHK(hipMemcpyAsync(dst, s->base + s->L.off_lo[s->fcur], s->L.plane * 4,
                              hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return LBM_OK;
}

lbm_status lbm_load(lbm_sim* s, const void* host, size_t bytes) {
    if (!s || !host) return fail(LBM_EINVAL, "null argument");
    if (bytes < lbm_state_bytes(s)) return fail(LBM_EINVAL, "buffer too small");
    CkptHeader h;
    std::memcpy(&h, host, sizeof(h));
    if (std::memcmp(h.magic, kCkptMagic, 8) != 0) return fail(LBM_EINVAL, "not a checkpoint");
    if (h.p.Nx != s->p.Nx || h.p.Ny != s->p.Ny || h.p.precision != s->p.precision ||
        (h.p.flags & LBM_PERIODIC_Y) != (s->p.flags & LBM_PERIODIC_Y))
        return fail(LBM_EINVAL, "checkpoint grid or precision differs");
    if (validate(h.p) != LBM_OK) return LBM_EINVAL;  // message set by validate
    HIPCHK(hipSetDevice(s->dev));
    HIPCHK(hipStreamSynchronize(s->stream));
    const char* src = static_cast<const char*>(host) + sizeof(h);
    const size_t fb = 9 * s->L.plane * s->L.esz, tb = s->L.plane * s->L.esz;
    HIPCHK(hipMemcpyAsync(s->base + s->L.off_f[s->fcur], src, fb, hipMemcpyHostToDevice, s->stream));
    src += fb;
    HIPCHK(hipMemcpyAsync(s->base + s->L.off_T[s->tcur], src, tb, hipMemcpyHostToDevice, s->stream));
    src += tb;
    if (s->p.precision == LBM_FP32_DEV_MASSEXACT)
        HIPCHK(hipMemcpyAsync(s->base + s->L.off_lo[s->fcur], src, s->L.plane * 4,
                              hipMemcpyHostToDevice, s->stream));
    // a new state: its health counters start from zero
    HIPCHK(hipMemsetAsync(s->stat(), 0, lbmhost::kStatWords * sizeof(unsigned long long),
                          s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    const int seg = s->seg_rows;
    s->p = h.p;
    s->n = h.n;
    set_phys(s);
    set_grid(s, seg);
    return LBM_OK;
}

lbm_status lbm_set_launch(lbm_sim* s, int32_t seg_rows) {
    if (!s) return fail(LBM_EINVAL, "null sim");
    set_grid(s, seg_rows > 0 ? seg_rows : default_seg_rows(s->p, s->L.rows));
    return LBM_OK;
}

lbm_status lbm_get_launch(const lbm_sim* s, int32_t* seg_rows, int32_t* waves) {
    if (!s) return fail(LBM_EINVAL, "null sim");
    if (seg_rows) *seg_rows = s->g.seg_rows;
    if (waves) *waves = s->g.n_units;
    return LBM_OK;
}

lbm_status lbm_autotune(lbm_sim* s, int32_t steps_per_trial, double* best_ms) {
    if (!s) return fail(LBM_EINVAL, "null sim");
    if (steps_per_trial < 1) steps_per_trial = 10;
    HIPCHK(hipSetDevice(s->dev));
    // snapshot the state on the device; every trial restarts from it
    const size_t fb = 9 * s->L.plane * s->L.esz, tb = s->L.plane * s->L.esz;
    const size_t lb = s->p.precision == LBM_FP32_DEV_MASSEXACT ? s->L.plane * 4 : 0;
    // the trial steps must not count towards the channel's health counters
    unsigned long long stat0[lbmhost::kStatWords];
    HIPCHK(hipMemcpyAsync(stat0, s->stat(), sizeof(stat0), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    char* snap = nullptr;
    HIPCHK(hipMalloc(reinterpret_cast<void**>(&snap), fb + tb + lb));
    const int64_t n0 = s->n;
    const int f0 = s->fcur, t0 = s->tcur;
    auto restore = [&]() -> hipError_t {
        s->n = n0;
        s->fcur = f0;
        s->tcur = t0;
        hipError_t e = hipMemcpyAsync(s->base + s->L.off_f[f0], snap, fb, hipMemcpyDeviceToDevice,
                                      s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->base + s->L.off_T[t0], snap + fb, tb, hipMemcpyDeviceToDevice,
                               s->stream);
        if (e == hipSuccess && lb)
            e = hipMemcpyAsync(s->base + s->L.off_lo[f0], snap + fb + tb, lb,
                               hipMemcpyDeviceToDevice, s->stream);
        return e;
    };
    hipError_t e = hipMemcpyAsync(snap, s->base + s->L.off_f[f0], fb, hipMemcpyDeviceToDevice,
                                  s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(snap + fb, s->base + s->L.off_T[t0], tb, hipMemcpyDeviceToDevice,
                           s->stream);
    if (e == hipSuccess && lb)
        e = hipMemcpyAsync(snap + fb + tb, s->base + s->L.off_lo[f0], lb, hipMemcpyDeviceToDevice,
                           s->stream);
    // segment heights with seg + 10 (the recomputed halo rows) a multiple of
    // the kernel's six-row unroll, so full segments need no padding rows
    std::vector<int> cands;
    for (int c = 2; c <= 128; c += 6)
        if (c <= s->L.rows) cands.push_back(c);
    for (int c : {152, 188, 248, 506})
        if (c <= s->L.rows) cands.push_back(c);
    cands.push_back(s->L.rows);
    cands.push_back(default_seg_rows(s->p, s->L.rows));
    std::sort(cands.begin(), cands.end());
    cands.erase(std::unique(cands.begin(), cands.end()), cands.end());
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
    double best = 1e300;
    int best_seg = s->seg_rows;
    for (size_t ci = 0; ci < cands.size() && e == hipSuccess; ++ci) {
        set_grid(s, cands[ci]);
        for (int w = 0; w < 2 && e == hipSuccess; ++w) e = enqueue_step(s);
        if (e == hipSuccess) e = hipEventRecord(ev0, s->stream);
        for (int i = 0; i < steps_per_trial && e == hipSuccess; ++i) e = enqueue_step(s);
        if (e == hipSuccess) e = hipEventRecord(ev1, s->stream);
        if (e == hipSuccess) e = hipEventSynchronize(ev1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
        if (e == hipSuccess && ms / steps_per_trial < best) {
            best = ms / steps_per_trial;
            best_seg = cands[ci];
        }
        if (e == hipSuccess) e = restore();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->stat(), stat0, sizeof(stat0), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    (void)hipFree(snap);
    set_grid(s, best_seg);
    if (e != hipSuccess) return fail(LBM_EDEVICE, "autotune: %s", hipGetErrorString(e));
    if (best_ms) *best_ms = best;
    return LBM_OK;
}

lbm_status lbm_bandwidth_probe(size_t bytes, int32_t iters, double* gbps, double* ms_per_copy) {
    if (bytes < 16 || iters < 1) return fail(LBM_EINVAL, "bytes >= 16 and iters >= 1 needed");
    bytes = bytes / 16 * 16;
    void *a = nullptr, *b = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&a, bytes);
    if (e == hipSuccess) e = hipMalloc(&b, bytes);
    if (e == hipSuccess) e = hipStreamCreate(&st);
    if (e == hipSuccess) e = hipMemsetAsync(a, 0, bytes, st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = lbmk::launch_copy(a, b, bytes, st);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int i = 0; i < iters && e == hipSuccess; ++i) e = lbmk::launch_copy(a, b, bytes, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (e != hipSuccess) return fail(LBM_EDEVICE, "bandwidth probe: %s", hipGetErrorString(e));
    const double per = ms / iters;
    if (gbps) *gbps = 2.0 * (double)bytes / (per * 1e-3) / 1e9;
    if (ms_per_copy) *ms_per_copy = per;
    return LBM_OK;
}

}  // extern "C"
