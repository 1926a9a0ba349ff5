// HIP kernels (gfx950 / CDNA4) of the pseudopotential MRT lattice Boltzmann
// step with the coupled RK4 temperature update, arXiv:1803.01756 Section 2.
//
// Fused step layout.  Populations are structure-of-arrays planes
// [9][rows][pitch] of deviations d_i = f_i - w_i rho_ref (x fastest, pitch a
// multiple of 64), temperature a plane [rows][pitch] of T - T_ref.  Only the
// fluid rows are stored.  The buffers hold post-collision values, so a step
// pulls f_i(x) = f*_i(x - e_i), or f*_opp(i)(x) where x - e_i is a plate
// (half-way bounce-back), and writes f*(x) in place of its own node into the
// other buffer of the A-B pair.
//
// Each wave owns a strip of 54 columns (lane l holds column strip*54 - 5 + l,
// periodic in x) and marches upward over a segment of fluid rows.  Neighbour
// columns come from the adjacent lanes through DPP wave shifts, neighbour rows
// from registers, so the whole step is one pass without LDS or barriers.  In
// the iteration whose leading row is k the wave
//   A  pulls row k and computes rho, j, psi(rho, T) there,
//   B  computes the forces, u and the MRT collision on row k-1,
//   C..F evaluate the RK4 stages h1..h4 on rows k-2 .. k-5,
// so every stage only needs rows that earlier stages of the same or previous
// iterations produced.  A stage loses one valid lane per side, hence the
// 5-column halo; rows of the halo above and below the segment are recomputed
// (5 extra leading and trailing iterations).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "lbm_internal.h"

namespace lbmk {
namespace {

constexpr uint32_t kFreezeT = 1u, kSinglePhase = 2u, kEosCS = 32u, kPhaseProps = 128u,
                   kTopMixed = 256u;

// ---- lane shifts (DPP wave_shr:1 / wave_shl:1) ---------------------------
// at_xm(v): the value lane l-1 holds (column x-1); at_xp: lane l+1 (x+1).  The
// edge lanes (which lie in the halo) read 0.
__device__ __forceinline__ int dpp_shr1(int v) {
    return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true);
}
__device__ __forceinline__ int dpp_shl1(int v) {
    return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true);
}
__device__ __forceinline__ float at_xm(float v) { return __int_as_float(dpp_shr1(__float_as_int(v))); }
__device__ __forceinline__ float at_xp(float v) { return __int_as_float(dpp_shl1(__float_as_int(v))); }
__device__ __forceinline__ double at_xm(double v) {
    int2 w = *reinterpret_cast<int2*>(&v);
    w.x = dpp_shr1(w.x);
    w.y = dpp_shr1(w.y);
    return *reinterpret_cast<double*>(&w);
}
__device__ __forceinline__ double at_xp(double v) {
    int2 w = *reinterpret_cast<int2*>(&v);
    w.x = dpp_shl1(w.x);
    w.y = dpp_shl1(w.y);
    return *reinterpret_cast<double*>(&w);
}

// A row value at x kept as the centre c, the x-sum a = v(x+1) + v(x-1) and
// the x-difference d = v(x+1) - v(x-1): every nine-point stencil of the
// step (Eq. 9 force, Eq. 16 gradient, Laplacian and divergence) uses only
// these three per row, computed once when the row is produced.
template <class R>
struct Tri {
    R c, a, d;
};
template <class R>
__device__ __forceinline__ Tri<R> tri(R v) {
    const R m = at_xm(v), p = at_xp(v);
    Tri<R> t;
    t.c = v;
    t.a = p + m;
    t.d = p - m;
    return t;
}
template <class R>
__device__ __forceinline__ Tri<R> tri_const(R v) {
    Tri<R> t;
    t.c = v;
    t.a = v + v;
    t.d = (R)0;
    return t;
}

// ---- raw buffer access ------------------------------------------------------
// The planes are addressed through buffer resources: a wave-uniform byte
// offset (plane and row, scalar register) plus a per-lane byte offset (the
// column), so a load or store needs no per-lane 64-bit address arithmetic.
// num_records is the buffer size, so an access outside it reads 0 / is
// dropped by the hardware range check.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kBufWord3 = 0x00020000;  // gfx9 raw-buffer format word

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kBufWord3);
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff, 0);
}

// A register copy the compiler cannot fold away: reading a loaded value here
// places the wait for its load at this point of the program.
__device__ __forceinline__ float settle(float v) {
    float r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

// A uniform value copied into a vector register (kept there by the compiler).
__device__ __forceinline__ float in_vgpr(float v) {
    float r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}
__device__ __forceinline__ double in_vgpr(double v) { return v; }

// ---- rows -----------------------------------------------------------------
struct RowK {
    bool fluid;   // stored fluid row
    bool bb_lo;   // the row below is a plate (bounce-back of e_y = +1 links)
    bool bb_hi;   // the row above is a plate
    int sr;       // stored row index
};
__device__ __forceinline__ RowK row_info(int y, const Grid& g) {
    RowK r;
    if (g.periodic_y) {
        int yy = y % g.Ny;
        if (yy < 0) yy += g.Ny;
        r.fluid = true;
        r.bb_lo = r.bb_hi = false;
        r.sr = yy;
        return r;
    }
    r.fluid = (y >= 1 && y <= g.Ny - 2);
    r.bb_lo = (y == 1);
    r.bb_hi = (y == g.Ny - 2);
    r.sr = y - 1;
    return r;
}

// Pull of Eq. 12 for one stored row: f_i(x) = f*_i(x - e_i) or, across a
// plate, f*_opp(i)(x).  Velocity order of Eq. 2: 0 rest, 1 +x, 2 +y, 3 -x,
// 4 -y, 5 (+,+), 6 (-,+), 7 (-,-), 8 (+,-).
template <class S>
__device__ __forceinline__ void pull_row(const S* __restrict__ f, const Grid& g, const RowK& r,
                                         unsigned x, unsigned xm, unsigned xp, S d[9]) {
    const unsigned P = g.plane, pitch = (unsigned)g.pitch;
    const unsigned rc = (unsigned)r.sr * pitch;
    unsigned rdn, rup;
    if (g.periodic_y) {
        int a = r.sr - 1, b = r.sr + 1;
        if (a < 0) a += g.rows;
        if (b >= g.rows) b -= g.rows;
        rdn = (unsigned)a * pitch;
        rup = (unsigned)b * pitch;
    } else {
        rdn = rc - pitch;
        rup = rc + pitch;
    }
    const unsigned o0 = rc + x;
    const unsigned o1 = P + rc + xm;
    const unsigned o3 = 3 * P + rc + xp;
    const unsigned o2 = r.bb_lo ? 4 * P + rc + x : 2 * P + rdn + x;
    const unsigned o5 = r.bb_lo ? 7 * P + rc + x : 5 * P + rdn + xm;
    const unsigned o6 = r.bb_lo ? 8 * P + rc + x : 6 * P + rdn + xp;
    const unsigned o4 = r.bb_hi ? 2 * P + rc + x : 4 * P + rup + x;
    const unsigned o7 = r.bb_hi ? 5 * P + rc + x : 7 * P + rup + xp;
    const unsigned o8 = r.bb_hi ? 6 * P + rc + x : 8 * P + rup + xm;
    d[0] = f[o0];
    d[1] = f[o1];
    d[2] = f[o2];
    d[3] = f[o3];
    d[4] = f[o4];
    d[5] = f[o5];
    d[6] = f[o6];
    d[7] = f[o7];
    d[8] = f[o8];
}

// The same pull through a buffer resource.  vx, vm, vp: byte offsets of the
// lane's columns x, x-1, x+1; the uniform scalar offset carries the buffer's
// offset from the resource base (fb) plus the plane and row.
template <class S>
__device__ __forceinline__ void pull_row_buf(__amdgpu_buffer_rsrc_t f, const Grid& g,
                                             const RowK& r, unsigned fb, unsigned vx,
                                             unsigned vm, unsigned vp, S d[9]) {
    const unsigned P = g.plane * (unsigned)sizeof(S), pitch = (unsigned)g.pitch * sizeof(S);
    const unsigned rc = fb + (unsigned)r.sr * pitch;
    unsigned rdn, rup;
    if (g.periodic_y) {
        int a = r.sr - 1, b = r.sr + 1;
        if (a < 0) a += g.rows;
        if (b >= g.rows) b -= g.rows;
        rdn = fb + (unsigned)a * pitch;
        rup = fb + (unsigned)b * pitch;
    } else {
        rdn = rc - pitch;
        rup = rc + pitch;
    }
    const S t = S(0);
    d[0] = bload(f, vx, rc, t);
    d[1] = bload(f, vm, P + rc, t);
    d[3] = bload(f, vp, 3 * P + rc, t);
    if (r.bb_lo) {
        d[2] = bload(f, vx, 4 * P + rc, t);
        d[5] = bload(f, vx, 7 * P + rc, t);
        d[6] = bload(f, vx, 8 * P + rc, t);
    } else {
        d[2] = bload(f, vx, 2 * P + rdn, t);
        d[5] = bload(f, vm, 5 * P + rdn, t);
        d[6] = bload(f, vp, 6 * P + rdn, t);
    }
    if (r.bb_hi) {
        d[4] = bload(f, vx, 2 * P + rc, t);
        d[7] = bload(f, vx, 5 * P + rc, t);
        d[8] = bload(f, vx, 6 * P + rc, t);
    } else {
        d[4] = bload(f, vx, 4 * P + rup, t);
        d[7] = bload(f, vp, 7 * P + rup, t);
        d[8] = bload(f, vm, 8 * P + rup, t);
    }
}

// ---- arithmetic helpers -------------------------------------------------------
// FP32: the hardware reciprocal and square root (about 1 ulp) replace the
// IEEE division / correctly rounded square root sequences.  FP64 (the FP64
// storage build) keeps IEEE division and sqrt.
__device__ __forceinline__ float rcp_r(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_r(double x) { return 1.0 / x; }
__device__ __forceinline__ float sqrt_r(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_r(double x) { return sqrt(x); }

// FP64 reciprocal and square root from the FP32 hardware estimates (relative
// error ~1e-7) refined by Newton steps, each squaring the error: two steps
// reach ~1 ulp of FP64 (the FP64 build), one step ~1e-14 relative, far below
// what FP32 storage resolves (the FP32 builds).
template <int kSteps>
__device__ __forceinline__ double rcp_d(double x) {
    double y = (double)__builtin_amdgcn_rcpf((float)x);
#pragma unroll
    for (int i = 0; i < kSteps; ++i) y = fma(y, fma(-x, y, 1.0), y);
    return y;
}
template <int kSteps>
__device__ __forceinline__ double sqrt_d(double x) {
    double y = (double)__builtin_amdgcn_rsqf((float)x);
    const double h = 0.5 * x;
#pragma unroll
    for (int i = 0; i < kSteps; ++i) y = y * fma(-h, y * y, 1.5);
    return x * y;
}

// Eqs. 10-11: psi = sqrt(2 (P_EOS(rho, T) - rho/3) / G), clamped at 0.
// FP64 throughout: the Shan-Chen force is a difference of neighbouring psi
// values and the FP32 rounding of psi itself would be of the order of that
// difference in a nearly uniform vapour.  With s = 1 + k (1 - sqrt(T/Tc)),
// D = 1 + 2 b rho - b^2 rho^2:
//   P = [rho R T D - a s^2 rho^2 (1 - b rho)] / ((1 - b rho) D).
// kF32: sqrt(T/Tc) in FP32 (its rounding enters phi as a smooth relative
// error, not a neighbour difference); the FP64 build takes it in FP64.
// The Carnahan-Starling option (flag kEosCS), e = b rho / 4:
//   P = rho R T (1 + e + e^2 - e^3) / (1 - e)^3 - a rho^2.
// kExt: the build that also serves the optional features (here the
// Carnahan-Starling EOS); the plain build leaves their code out.
// clamped: set when the argument is not positive (psi is then 0), the event
// the step counts per owned node.
template <bool kF32, bool kExt = true>
__device__ __forceinline__ double psi_eos(double rho, double T, const Phys& k, bool& clamped) {
    constexpr int kNewton = kF32 ? 1 : 2;
    if (kExt && (k.flags & kEosCS)) {
        const double e = 0.25 * k.b * rho, o = 1.0 - e;
        const double Z = (1.0 + e * (1.0 + e * (1.0 - e))) * rcp_d<kNewton>(o * o * o);
        const double P = rho * (k.R * T * Z - k.a * rho);
        const double arg = 2.0 * (P - rho * (1.0 / 3.0)) * k.inv_G;
        clamped = !(arg > 0.0);
        return arg > 0.0 ? sqrt_d<kNewton>(arg) : 0.0;
    }
    const double st = kF32 ? (double)__builtin_amdgcn_sqrtf((float)(T * k.inv_Tc))
                           : sqrt_d<2>(T * k.inv_Tc);
    const double s = 1.0 + k.kappa * (1.0 - st);
    const double br = k.b * rho;
    const double omb = 1.0 - br;
    const double D = 1.0 + br * (2.0 - br);
    const double num = rho * (k.R * T * D - k.a * (s * s) * rho * omb);
    const double P = num * rcp_d<kNewton>(omb * D);
    const double arg = 2.0 * (P - rho * (1.0 / 3.0)) * k.inv_G;
    clamped = !(arg > 0.0);
    return arg > 0.0 ? sqrt_d<kNewton>(arg) : 0.0;
}

// Eq. 9 + Eq. 14 in one sum: the solid rows carry the effective potential
// psi_w G_w / G, so -G psi(x) sum_i w_i phi(x + e_i) e_i is F_m + F_ads.
__device__ __forceinline__ void pair_force(const Tri<double>& pS, const Tri<double>& pC,
                                           const Tri<double>& pN, double negG, double& Fx,
                                           double& Fy) {
    const double sx = pC.d * (1.0 / 3.0) + (pN.d + pS.d) * (1.0 / 12.0);
    const double sy = (pN.c - pS.c) * (1.0 / 3.0) + (pN.a - pS.a) * (1.0 / 12.0);
    Fx = negG * pC.c * sx;
    Fy = negG * pC.c * sy;
}

// Eq. 14 alone on the first / last fluid row: the three links crossing a
// plate carry weight 1/3 + 2/12 = 1/2.
__device__ __forceinline__ double wall_adhesion_y(const RowK& r, double psi_c, const Phys& k) {
    double f = 0.0;
    if (r.bb_lo) f += 0.5 * k.Gw_psiw * psi_c;
    if (r.bb_hi) f -= 0.5 * k.Gw_psiw * psi_c;
    return f;
}

template <class R>
__device__ __forceinline__ const PhysR<R>& pr(const Phys& k);
template <>
__device__ __forceinline__ const PhysR<float>& pr<float>(const Phys& k) { return k.rf; }
template <>
__device__ __forceinline__ const PhysR<double>& pr<double>(const Phys& k) { return k.rd; }

// MRT collision, Eqs. 6-8, in deviation moments: m'_k = m_k - rho_ref (M w)_k.
// Returns the post-collision deviations in d (overwritten).
template <class R>
__device__ __forceinline__ void collide(R d[9], R drho, R rho, R rinv, R ux, R uy, R Fx, R Fy,
                                        R th, R sv, const PhysR<R>& c) {
    const R s_rho = c.s_rho, s_e = c.s_e, s_z = c.s_z, s_j = c.s_j, s_q = c.s_q;
    const R axis = (d[1] + d[2]) + (d[3] + d[4]);
    const R diag = (d[5] + d[6]) + (d[7] + d[8]);
    R m[9];
    m[0] = drho;
    m[1] = (R)-4 * d[0] - axis + (R)2 * diag;
    m[2] = (R)4 * d[0] - (R)2 * axis + diag;
    m[3] = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
    m[4] = (R)2 * (d[3] - d[1]) + (d[5] - d[6]) + (d[8] - d[7]);
    m[5] = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
    m[6] = (R)2 * (d[4] - d[2]) + (d[5] + d[6]) - (d[7] + d[8]);
    m[7] = (d[1] + d[3]) - (d[2] + d[4]);
    m[8] = (d[5] + d[7]) - (d[6] + d[8]);
    const R jx = rho * ux, jy = rho * uy;
    const R j2r = (jx * jx + jy * jy) * rinv;
    R meq[9];
    meq[0] = drho;
    meq[1] = (R)-2 * drho + (R)3 * j2r;
    meq[2] = drho - (R)3 * j2r;
    meq[3] = jx;
    meq[4] = -jx;
    meq[5] = jy;
    meq[6] = -jy;
    meq[7] = (jx * jx - jy * jy) * rinv;
    meq[8] = jx * jy * rinv;
    const R uF = ux * Fx + uy * Fy;
    R S[9];
    S[0] = (R)0;
    S[1] = (R)6 * uF + c.c_e * th;
    S[2] = (R)-6 * uF - c.c_z * th;
    S[3] = Fx;
    S[4] = -Fx;
    S[5] = Fy;
    S[6] = -Fy;
    S[7] = (R)2 * (ux * Fx - uy * Fy);
    S[8] = ux * Fy + uy * Fx;
    const R s[9] = {s_rho, s_e, s_z, s_j, s_q, s_j, s_q, sv, sv};
    R a[9];
    const R nrm[9] = {(R)1 / 9, (R)1 / 36, (R)1 / 36, (R)1 / 6, (R)1 / 12,
                      (R)1 / 6, (R)1 / 12, (R)1 / 4, (R)1 / 4};
#pragma unroll
    for (int q = 0; q < 9; ++q)
        a[q] = (m[q] - s[q] * (m[q] - meq[q]) + ((R)1 - (R)0.5 * s[q]) * S[q]) * nrm[q];
    // conserved moments: m*_0 = m_0 and, since m_eq3 = m_3 + F_x / 2 (the
    // velocity holds half the force), m*_3 = m_3 + F_x and m*_5 = m_5 + F_y
    // for any rate; written directly, the rates s_rho and s_j drop out
    a[0] = drho * nrm[0];
    a[3] = (m[3] + Fx) * nrm[3];
    a[5] = (m[5] + Fy) * nrm[5];
    // f* = M^T diag(1/|M_k|^2) m*
    const R b0 = a[0] - a[1] - (R)2 * a[2];
    const R c0 = a[0] + (R)2 * a[1] + a[2];
    d[0] = a[0] - (R)4 * a[1] + (R)4 * a[2];
    d[1] = b0 + a[3] - (R)2 * a[4] + a[7];
    d[2] = b0 + a[5] - (R)2 * a[6] - a[7];
    d[3] = b0 - a[3] + (R)2 * a[4] + a[7];
    d[4] = b0 - a[5] + (R)2 * a[6] - a[7];
    d[5] = c0 + a[3] + a[4] + a[5] + a[6] + a[8];
    d[6] = c0 - a[3] - a[4] + a[5] + a[6] - a[8];
    d[7] = c0 - a[3] - a[4] - a[5] - a[6] + a[8];
    d[8] = c0 + a[3] + a[4] - a[5] - a[6] - a[8];
}

// Per-row coefficients of K(T) (Eq. 16) with rho(n), u(n) frozen:
//   K = -(u . grad T) + q3 lap T - q1 T - q2 sqrt(T),
// using T (dP/dT)_rho = (A - B2) T + B1 sqrt(T), A = rho R / (1 - b rho),
// B1 = a k (1 + k) rho^2 / (sqrt(Tc) D), B2 = a k^2 rho^2 / (Tc D),
// D = 1 + 2 b rho - b^2 rho^2, and c = 1 / (rho C_v):
//   q1 = c div(u) (A - B2), q2 = c div(u) B1, q3 = c lambda.
// FP32 build: an RK stage moves T by ~1e-4 relative, so sqrt(T) is taken
// linear about the row's T(n): sqrt(T) = s + (T - T_n)/(2 s), s = sqrt(T_n)
// (neglected term (T - T_n)^2 / (8 s^3), ~1e-9 relative), which turns the
// last two terms into -Q1 T - Q0 with Q1 = q1 + q2/(2 s), Q0 = q2 s / 2 and
// needs one reciprocal square root per row instead of one square root per
// stage; with T = T_ref + t (stored deviation) the constant becomes
// Q0 + Q1 T_ref.  The FP64 build keeps the exact sqrt.
template <class R>
struct Coef {
    R ux, uy, q1, q2, q3;
};
// lam_c, glx, gly, inv_cv: the conductivity at the node, its gradient and
// 1/C_v (constants unless lambda and C_v depend on the phase).  The
// conduction term [lambda lap T + grad(lambda).grad(T)] / (rho C_v) is
// carried as q3 lap T plus a shift of the advecting velocity by
// -grad(lambda) / (rho C_v).  amax > 0: where the diffusivity
// lambda / (rho C_v) exceeds amax the whole conduction term is scaled by
// amax over it (a departure from Eq. 17 that keeps the explicit RK4 of the
// conduction term inside its stability bound in thin vapour).
template <class R>
__device__ __forceinline__ Coef<R> heat_coef(R rho, R ux, R uy, R divu, R Tn, R T_ref,
                                             const PhysR<R>& pc, bool cs, bool props,
                                             R lam_c, R glx, R gly, R inv_cv, R amax) {
    R A, r2D, c;
    if (cs) {
        // Carnahan-Starling: T (dP/dT)_rho = rho R Z(e) T, no sqrt(T) term
        // (rkB1 = rkB2 = 0); inv = 1 / ((1 - e)^3 rho)
        const R e = (R)0.25 * pc.b * rho, o = (R)1 - e, o3 = o * o * o;
        const R inv = rcp_r(o3 * rho);
        A = rho * rho * pc.rkA * ((R)1 + e * ((R)1 + e * ((R)1 - e))) * inv;
        r2D = 0;
        c = (props ? inv_cv : pc.inv_Cv) * o3 * inv;
    } else {
        const R br = pc.b * rho;
        const R omb = (R)1 - br;
        const R D = (R)1 + br * ((R)2 - br);
        const R inv = rcp_r(omb * D * rho);  // 1 / ((1 - b rho) D rho)
        A = rho * rho * pc.rkA * D * inv;
        r2D = rho * rho * rho * omb * inv;
        c = (props ? inv_cv : pc.inv_Cv) * omb * D * inv;
    }
    Coef<R> q;
    const R lam = props ? lam_c : pc.lambda;
    R cg = c;  // 1 / (rho C_v) as the conduction term sees it
    q.q3 = c * lam;
    if (amax > (R)0 && q.q3 > amax) {
        cg = amax * rcp_r(lam);
        q.q3 = amax;
    }
    q.ux = props ? ux - cg * glx : ux;
    q.uy = props ? uy - cg * gly : uy;
    q.q1 = c * divu * (A - pc.rkB2 * r2D);
    q.q2 = c * divu * pc.rkB1 * r2D;
    if (sizeof(R) == 4) {
        const R rs = (R)__builtin_amdgcn_rsqf((float)Tn);  // 1 / sqrt(T_n)
        const R sn = Tn * rs;
        q.q1 = q.q1 + q.q2 * (R)0.5 * rs;             // Q1
        q.q2 = q.q2 * (R)0.5 * sn + q.q1 * T_ref;     // Q0 + Q1 T_ref
    }
    return q;
}

// K(T) on the stage field (deviations tS, tC, tN of rows y-1, y, y+1).
template <class R>
__device__ __forceinline__ R heat_rhs(const Tri<R>& tS, const Tri<R>& tC, const Tri<R>& tN,
                                      const Coef<R>& q, R T_ref) {
    const R third = (R)1 / 3, twelfth = (R)1 / 12;
    const R tx = tC.d * third + (tN.d + tS.d) * twelfth;
    const R ty = (tN.c - tS.c) * third + (tN.a - tS.a) * twelfth;
    const R ax = tC.a + (tN.c + tS.c);
    const R dg = tN.a + tS.a;
    const R lap = ax * ((R)2 / 3) + dg * ((R)1 / 6) - tC.c * ((R)10 / 3);
    const R adv_cond = -(q.ux * tx + q.uy * ty) + q.q3 * lap;
    if (sizeof(R) == 4) return adv_cond - q.q1 * tC.c - q.q2;
    const R Tabs = T_ref + tC.c;
    return adv_cond - q.q1 * Tabs - q.q2 * sqrt_r(Tabs);
}

// divergence of u at row y from rows y-1 (uS), y (uC), y+1 (uN)
template <class R>
__device__ __forceinline__ R div_u(const Tri<R>& xS, const Tri<R>& xC, const Tri<R>& xN,
                                   const Tri<R>& yS, const Tri<R>& yC, const Tri<R>& yN) {
    const R third = (R)1 / 3, twelfth = (R)1 / 12;
    return (xC.d + (yN.c - yS.c)) * third + ((xN.d + xS.d) + (yN.a - yS.a)) * twelfth;
}

template <class S>
struct RealOf;
template <>
struct RealOf<float> {
    using T = float;
};
template <>
struct RealOf<double> {
    using T = double;
};

// Open ends: the inlet density at time level n, the vapour-branch root of
// P_EOS(rho, T_in) = p0 (1 + p_amp sin(2 pi n / p_period)) (constant
// p0 (1 + p_amp) when p_period <= 0).  Safeguarded Newton from rho_v inside
// (0, rho_sp), rho_sp the vapour spinodal: a fixed number of iterations, so
// a channel gets the same bits alone and in a batch.
__device__ double inlet_density(const Phys& k, long long n) {
    const double T = k.T_in_eos;
    const double target = k.p_period > 0.0
        ? k.p0 * (1.0 + k.p_amp * sin(2.0 * 3.14159265358979323846 * (double)n / k.p_period))
        : k.p0 * (1.0 + k.p_amp);
    const bool cs = (k.flags & kEosCS) != 0;
    const double s = 1.0 + k.kappa * (1.0 - sqrt(T * k.inv_Tc));
    const double aphi = k.a * s * s;
    double lo = 0.0, hi = k.rho_sp, r = k.rho_v;
    for (int it = 0; it < 60; ++it) {
        double P, dP;
        if (cs) {
            const double e = 0.25 * k.b * r, o = 1.0 - e, o3 = o * o * o;
            P = r * k.R * T * (1.0 + e * (1.0 + e * (1.0 - e))) / o3 - k.a * r * r;
            dP = k.R * T * (1.0 + e * (4.0 + e * (4.0 + e * (-4.0 + e)))) / (o3 * o) -
                 2.0 * k.a * r;
        } else {
            const double br = k.b * r, omb = 1.0 - br, D = 1.0 + br * (2.0 - br);
            P = r * k.R * T / omb - aphi * r * r / D;
            dP = k.R * T / (omb * omb) - 2.0 * aphi * r * (1.0 + br) / (D * D);
        }
        if (P < target) lo = r; else hi = r;
        double rn = r - (P - target) / dP;
        if (!(rn > lo && rn < hi)) rn = 0.5 * (lo + hi);
        r = rn;
    }
    return r;
}

// Zou-He on an open end (zero transverse velocity, prescribed density), in
// deviations d_i = f_i - w_i rho_ref (the rho_ref parts cancel): with
// J = rho u_x from the known populations, the inlet (x = 0) rebuilds d1, d5,
// d8, the outlet (x = Nx-1, density rho_v) d3, d6, d7.  A corner node (next
// to a plate) takes the velocity form with u = 0 (J = 0).
template <class R>
__device__ __forceinline__ void zou_he(R d[9], bool at_in, bool at_out, double rho_in,
                                       const Phys& k, bool corner) {
    const R dd = (R)0.5 * (d[2] - d[4]);
    if (at_in) {
        R J = (R)(rho_in - k.rho_ref) - (d[0] + d[2] + d[4] + (R)2 * (d[3] + d[6] + d[7]));
        if (corner) J = 0;
        d[1] = d[3] + J * ((R)2 / 3);
        d[5] = d[7] - dd + J * ((R)1 / 6);
        d[8] = d[6] + dd + J * ((R)1 / 6);
    }
    if (at_out) {
        R J = (R)(k.rho_ref - k.rho_v) + (d[0] + d[2] + d[4] + (R)2 * (d[1] + d[5] + d[8]));
        if (corner) J = 0;
        d[3] = d[1] - J * ((R)2 / 3);
        d[7] = d[5] + dd - J * ((R)1 / 6);
        d[6] = d[8] - dd - J * ((R)1 / 6);
    }
}

// Oscillating drive at time level n, evaluated on the device so that a channel
// run alone and inside a batch sees the same bits.
__device__ __forceinline__ double drive_at(const Phys& k, long long n) {
    return k.period > 0.0 ? k.g_osc * sin(2.0 * 3.14159265358979323846 * (double)n / k.period)
                          : 0.0;
}

// XCD-aware unit index: blocks are dispatched round-robin over the eight
// XCDs, so consecutive units (neighbouring strips, which share halo columns)
// are mapped to blocks that land on the same XCD and its L2.
__device__ __forceinline__ int unit_of_block(int nblocks_pad) {
    const int b = blockIdx.x;
    const int per = nblocks_pad >> 3;
    return ((b & 7) * per + (b >> 3));
}

// Add a wave's health word (see step_unit) to the counters: stat[0] gains
// the number of lanes (node columns of the segment) that read a non-finite
// value, stat[1] the clamped Eq. 10 arguments.  Called by every lane of the
// wave; the sums and the atomics run only when some lane counted anything.
__device__ __forceinline__ void flush_health(unsigned long long* stat, unsigned health) {
    if (__builtin_amdgcn_ballot_w64(health != 0u) == 0ull) return;
    const unsigned long long bad = __builtin_amdgcn_ballot_w64((health >> 31) != 0u);
    unsigned clamp = health & 0x7fffffffu;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) clamp += __shfl_xor(clamp, off, 64);
    if ((threadIdx.x & (kLanes - 1)) == 0) {
        if (bad) atomicAdd(&stat[0], (unsigned long long)__builtin_popcountll(bad));
        if (clamp) atomicAdd(&stat[1], (unsigned long long)clamp);
    }
}

// One wave's share of a step: the strip and row segment of `unit`.  kExt
// compiles in the optional features (held and reservoir frames, the
// Carnahan-Starling EOS, open ends and plate temperature ramps,
// phase-dependent conductivity and heat capacity, the Sec. 3.2 plates); the
// plain instantiation, used whenever none is set, keeps the register budget
// of three waves per SIMD.
template <class S, bool kMX, bool kExt>
__device__ __forceinline__ void step_unit(const Grid& g, const Phys& k, const Bufs<S>& B,
                                          double drive, double rho_in, int unit) {
    using R = typename RealOf<S>::T;
    const int lane = threadIdx.x & (kLanes - 1);
    const int strip = unit % g.n_strips;
    const int seg = unit / g.n_strips;

    // lane column and its periodic neighbours
    int cx = strip * kOwned - kHalo + lane;
    cx %= g.Nx;
    if (cx < 0) cx += g.Nx;
    const unsigned x = (unsigned)cx;
    const unsigned xm = (unsigned)(cx == 0 ? g.Nx - 1 : cx - 1);
    const unsigned xp = (unsigned)(cx == g.Nx - 1 ? 0 : cx + 1);
    const int own_w = min(kOwned, g.Nx - strip * kOwned);
    const bool own_lane = lane >= kHalo && lane < kHalo + own_w;
    // Lanes that store post-collision populations.  The collision is exact
    // on every lane but the outermost one of each side (its force needs psi
    // one column past the wave), so a wave holds its neighbours' first four
    // columns exactly.  A boundary between two strips that would split a
    // 64-byte chunk of a row into a part of at most four columns and the
    // rest is moved so that one wave writes the whole chunk: a row store then
    // makes fewer partial-chunk write requests, and every column is still
    // written by exactly one wave.  Rows start on 64-byte boundaries.  T(n+1)
    // is exact on the owned lanes only and keeps them.
    const int c0 = strip * kOwned;
    auto moved = [&](const int b, const int b_next) {
        constexpr int cpc = 64 / (int)sizeof(S), kMove = kHalo - 1;
        const int r = b % cpc;
        if (r == 0) return b;
        if (r <= kMove) return b - r;
        if (cpc - r <= kMove && b + (cpc - r) <= b_next) return b + (cpc - r);
        return b;
    };
    const int st_lo = strip > 0 ? moved(c0, c0 + own_w) : 0;
    const int st_hi = strip + 1 < g.n_strips ? moved(c0 + kOwned, min(c0 + 2 * kOwned, g.Nx))
                                             : c0 + own_w;
    const bool store_lane = c0 - kHalo + lane >= st_lo && c0 - kHalo + lane < st_hi;
    // Lane masks and the register budget (each choice measured on 8192 x
    // 512): the FP64 and mass-exact builds count each node's health on the
    // lanes that store it, beside the stores; the FP64 build, shortest of
    // scalar registers, also tests the owned lanes only where T(n+1) is
    // stored, so that a single mask stays live through its row loop.  The
    // plain FP32 build counts health on the owned lanes in a block of its
    // own.
    constexpr bool kHealthOnStore = sizeof(S) == 8 || kMX;
    constexpr bool kOwnedTestAtT = sizeof(S) == 8;
    // The frame of a box: the outermost columns, and in a periodic box the
    // outermost rows.  FRAME_T holds its temperature (the RK right-hand
    // sides are zeroed there); FRAME_RHO makes it a reservoir at rest
    // (rho = rho_frame, u = 0, post-collision populations the rest
    // equilibrium of rho_frame).
    const bool edge_col = cx == 0 || cx == g.Nx - 1;
    auto on_frame = [&](const RowK& r) {
        return edge_col || (g.periodic_y && (r.sr == 0 || r.sr == g.rows - 1));
    };
    // Open ends (OPEN_X): the inlet column holds T = T_in (the outlet column
    // T = T_out when it is held), stencils past the ends see the end
    // column's own value (zero-gradient ghost), and the plates may carry a
    // temperature linear in x.
    const bool open_x = kExt && g.open_x != 0;
    const bool at_in = open_x && cx == 0, at_out = open_x && cx == g.Nx - 1;
    const bool out_held = at_out && k.hold_out != 0;
    auto held = [&](const RowK& r) {
        return (kExt && g.frame_t && on_frame(r)) || at_in || out_held;
    };
    auto trix = [&](auto v) {
        if (!open_x) return tri(v);
        auto m = at_xm(v), p = at_xp(v);
        if (at_in) m = v;
        if (at_out) p = v;
        decltype(tri(v)) t;
        t.c = v;
        t.a = p + m;
        t.d = p - m;
        return t;
    };
    const bool ramp = kExt && k.wall_ramp != 0;
    const R dTw_x = ramp ? (R)(k.dT_wall + (k.dT_w_end - k.dT_wall) * (double)cx / (double)(g.Nx - 1))
                         : (R)k.dT_wall;
    auto wall_t = [&]() { return ramp ? trix(dTw_x) : tri_const<R>(pr<R>(k).dT_wall); };
    const bool frame_rho = kExt && g.frame_rho != 0;
    const bool props = kExt && (k.flags & kPhaseProps) != 0;
    const bool eos_cs = kExt && (k.flags & kEosCS) != 0;

    const int ya = g.y_first + seg * g.seg_rows;
    const int yb = min(ya + g.seg_rows, g.y_first + g.rows);

    const bool freezeT = (k.flags & kFreezeT) != 0;
    const bool single = (k.flags & kSinglePhase) != 0;
    const PhysR<R>& kr_ = pr<R>(k);
    // The collision and heat constants of the FP32 builds live in vector
    // registers: the scalar registers are short (the loop holds the FP64 EOS
    // constants, offsets and row state), and a vector operation reads at
    // most one scalar operand.
    PhysR<R> cv = kr_;
    if (sizeof(R) == 4) {
        cv.s_e = in_vgpr(cv.s_e);
        cv.s_z = in_vgpr(cv.s_z);
        cv.s_q = in_vgpr(cv.s_q);
        cv.c_e = in_vgpr(cv.c_e);
        cv.c_z = in_vgpr(cv.c_z);
        cv.b = in_vgpr(cv.b);
        cv.rkA = in_vgpr(cv.rkA);
        cv.rkB1 = in_vgpr(cv.rkB1);
        cv.rkB2 = in_vgpr(cv.rkB2);
        cv.inv_Cv = in_vgpr(cv.inv_Cv);
        cv.lambda = in_vgpr(cv.lambda);
    }
    const R T_ref = kr_.T_ref;
    const R dTw = kr_.dT_wall;
    const R rho_ref = kr_.rho_ref;
    // Sec. 3.2 plates (TOP_MIXED): the bottom plate holds its own
    // temperature; the top plate holds T_w on the cold columns and elsewhere
    // mirrors the fluid row below it, stage by stage (zero normal gradient
    // at the half-way wall).  plate_t: a plate row's stage value, given the
    // same stage's value of the row below.
    const bool top_mixed = kExt && (k.flags & kTopMixed) != 0;
    const bool adiab = top_mixed && !(cx >= k.cold_x0 && cx < k.cold_x1);
    auto plate_t = [&](const int y, const R below) {
        if (!top_mixed) return wall_t();
        if (y <= 0) return tri_const<R>((R)k.dT_w_bot);
        return trix(adiab ? below : dTw);
    };
    const R drive_r = (R)drive;

    // ---- register row windows ----
    // pulled deviations and derived values of rows k (cur) and k-1 (prv)
    R dPrv[9], dCur[9];
    R rhoCur = 0, rhoPrv = 0, rhoP2 = 0;  // rho of rows k, k-1, k-2
    R drCur = 0, drPrv = 0;
    R jxCur = 0, jyCur = 0, jxPrv = 0, jyPrv = 0;
    Tri<double> psi0, psi1, psi2;  // rows k, k-1, k-2
    // T(n) deviations: rows k .. k-5 (centre), shifted copies for rows k .. k-3
    Tri<R> tn0, tn1, tn2, tn3;
    R tn4 = 0, tn5 = 0;
    // velocity rows k-1, k-2, k-3
    Tri<R> ux1, ux2, ux3, uy1, uy2, uy3;
    // heat coefficients rows k-2 .. k-5
    Coef<R> cf2, cf3, cf4, cf5;
    // phase-dependent conductivity (optional): rows k-1, k-2, k-3
    Tri<R> lam1, lam2, lam3;
    // RK stage fields: T1 rows k-2..k-4, T2 rows k-3..k-5, T3 rows k-4..k-6
    Tri<R> t1a, t1b, t1c, t2a, t2b, t2c, t3a, t3b, t3c;
    R acc2 = 0, acc3 = 0, acc4 = 0, acc5 = 0;  // sum of the h's, rows k-2 .. k-5
    double drdCur = 0.0, drdPrv = 0.0;         // mass-exact: FP64 deviation density
    // health of the owned nodes (the state at level n), in one register:
    // bits 0-30 count the Eq. 10 arguments clamped to psi = 0 (a lane owns
    // fewer than 2^20 rows), bit 31 is set once the lane has read a
    // non-finite rho or T
    unsigned health = 0;

#pragma unroll
    for (int q = 0; q < 9; ++q) dPrv[q] = dCur[q] = 0;
    psi0 = psi1 = psi2 = tri_const<double>(0.0);
    tn0 = tn1 = tn2 = tn3 = tri_const<R>(dTw);
    ux1 = ux2 = ux3 = uy1 = uy2 = uy3 = tri_const<R>(0);
    cf2 = cf3 = cf4 = cf5 = Coef<R>{0, 0, 0, 0, 0};
    lam1 = lam2 = lam3 = tri_const<R>((R)k.lambda);
    t1a = t1b = t1c = t2a = t2b = t2c = t3a = t3b = t3c = tri_const<R>(dTw);

    // One buffer resource covers every buffer of the step (they share one
    // allocation); the lane's byte offset is its column, the uniform scalar
    // offset the buffer, plane and row.
    const unsigned esz = (unsigned)sizeof(S);
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(B.base, B.span);
    const unsigned vx = x * esz, vm = xm * esz, vp = xp * esz, vlo = x * 4u;
    const unsigned rowb = (unsigned)g.pitch * esz, rowb_lo = (unsigned)g.pitch * 4u;
    const unsigned P = g.plane * esz;

    // One row iteration; the loop below calls it six times per trip so that
    // the row windows of depth 2, 3 and 6 rotate by renaming registers instead
    // of moving them (a loop holding DPP operations is not unrolled by the
    // compiler); the depth-4 windows move once per trip.  Launch shapes with
    // seg_rows + 10 a multiple of 6 need no padding iterations.
    const int kr_end = yb + kHalo;
    // FP32 builds load row kr+1 at the top of iteration kr and move it into
    // the registers stage A reads (cur) later in the iteration (take_row
    // below: before the population stores or before the last stage), so the
    // loads overlap most of an iteration and the wait for them does not wait
    // for the stores that follow it (one counter tracks both).  Every
    // iteration loads: a row that is not a stored fluid row of the segment's
    // range reads the first stored row instead (values never used).  The
    // FP64 build (twice the registers per value) loads each row in stage A
    // of its own iteration.
    constexpr bool kAhead = sizeof(S) == 4;
    struct RawRow {
        S d[9];
        S T;
        float lo;
    };
    RawRow raw, cur;
    auto issue_loads = [&](const int y, RawRow& dst) {
        const RowK rL = row_info(y, g);
        const RowK rS = (rL.fluid && y < kr_end) ? rL : row_info(g.y_first, g);
        pull_row_buf<S>(rb, g, rS, B.fin, vx, vm, vp, dst.d);
        dst.T = bload(rb, vx, B.Tin + (unsigned)rS.sr * rowb, S(0));
        dst.lo = kMX ? bload(rb, vlo, B.lo_in + (unsigned)rS.sr * rowb_lo, 0.0f) : 0.0f;
    };
    // the loads of an interior row (plate-free neighbours, no wrap in y)
    auto issue_loads_interior = [&](const int y, RawRow& dst) {
        const RowK rL{true, false, false, y - 1};
        pull_row_buf<S>(rb, g, rL, B.fin, vx, vm, vp, dst.d);
        dst.T = bload(rb, vx, B.Tin + (unsigned)rL.sr * rowb, S(0));
        dst.lo = kMX ? bload(rb, vlo, B.lo_in + (unsigned)rL.sr * rowb_lo, 0.0f) : 0.0f;
    };
    if (kAhead) {
        issue_loads(ya - kHalo, raw);
        cur = raw;
    }
    // row kr+1 into the registers of the next iteration
    auto take_row = [&]() {
#pragma unroll
        for (int q = 0; q < 9; ++q) cur.d[q] = settle(raw.d[q]);
        cur.T = settle(raw.T);
        if (kMX) cur.lo = settle(raw.lo);
    };
    // Where the interior iteration takes its loaded row: just before the
    // population stores in the plain FP32 build (measured faster there), just
    // before the last stage otherwise (the mass-exact build measured slower
    // with the early wait).
    constexpr bool kEarlySettle = kAhead && !kMX;
    // A row iteration in two builds.  The general one (kFast false) handles
    // every case.  The interior one serves the steady state of a segment in
    // the common configuration (plates, temperature on, two phases, no
    // optional feature): every stage is active, all six rows are fluid rows
    // off the plates and the two stores are owned, so it has no branch but
    // the lane masks of the stores, which lets the scheduler interleave the
    // stages.
    auto row_interior = [&](const int kr, const int j) { return RowK{true, false, false, kr - j - 1}; };
    auto row_iteration = [&](const int kr, auto fast_tag) {
        constexpr bool kFast = decltype(fast_tag)::value;
        // Padding iterations past kr_end compute and store nothing.
        const bool live = kFast || kr < kr_end;
        if (kAhead) {
            if (kFast) issue_loads_interior(kr + 1, raw);
            else issue_loads(kr + 1, raw);
        }
        // ------------- stage A: row kr: pull, rho, j, psi -----------------
        const RowK rA = kFast ? row_interior(kr, 0) : row_info(kr, g);
        Tri<double> psiA;
        R dTA;
        if (kFast || (rA.fluid && live)) {
            if (!kAhead) issue_loads(kr, cur);
            const S rawT = cur.T;
            const R lo = kMX ? (R)cur.lo : (R)0;
#pragma unroll
            for (int q = 0; q < 9; ++q) dCur[q] = (R)cur.d[q];
            if (open_x) zou_he<R>(dCur, at_in, at_out, rho_in, k, rA.bb_lo || rA.bb_hi);
            double drd;
            if (kMX) {
                drd = (double)dCur[0] + (double)lo;
#pragma unroll
                for (int q = 1; q < 9; ++q) drd += (double)dCur[q];
            } else {
                R s = ((dCur[0] + dCur[1]) + (dCur[2] + dCur[3])) +
                      ((dCur[4] + dCur[5]) + (dCur[6] + dCur[7])) + dCur[8];
                drd = (double)s;
            }
            jxCur = (dCur[1] - dCur[3]) + (dCur[5] - dCur[6]) + (dCur[8] - dCur[7]);
            jyCur = (dCur[2] - dCur[4]) + (dCur[5] + dCur[6]) - (dCur[7] + dCur[8]);
            if (frame_rho && on_frame(rA)) {
                drd = k.rho_frame - k.rho_ref;
                jxCur = jyCur = 0;
            }
            drCur = (R)drd;
            drdCur = drd;
            const double rho_d = k.rho_ref + drd;
            rhoCur = (R)rho_d;
            dTA = (R)rawT;
            const double Td = k.T_ref + (double)dTA;
            bool clamped;
            psiA = trix(psi_eos<sizeof(S) == 4, kExt>(rho_d, Td, k, clamped));
        } else {
            drCur = 0;
            drdCur = 0.0;
            rhoCur = rho_ref;
            jxCur = jyCur = 0;
            dTA = ramp ? dTw_x : dTw;
            if (top_mixed) dTA = kr <= 0 ? (R)k.dT_w_bot : (adiab ? tn1.c : dTw);
            psiA = tri_const<double>(k.psi_wall_eff);
        }
        psi0 = psiA;
        tn0 = trix(dTA);

        // Stages whose row lies below the rows the segment needs from them are
        // skipped (the first iterations of a segment): B needs rows from
        // ya-4, C from ya-3, D from ya-2, E from ya-1 (each stage widens the
        // stencil by one row); their window entries are then never read.
        const bool needB = kFast || (live && kr - 1 >= ya - 4);
        const bool needC = kFast || (live && kr - 2 >= ya - 3);
        const bool needD = kFast || (live && kr - 3 >= ya - 2);
        const bool needE = kFast || (live && kr - 4 >= ya - 1);
        // ------------- stage B: forces, u, collision on row kr-1 ---------
        const RowK rB = kFast ? row_interior(kr, 1) : row_info(kr - 1, g);
        Tri<R> uxB, uyB;
        if (kFast || (rB.fluid && needB)) {
            double Fxd = 0.0, Fyd = 0.0, Fmx = 0.0, Fmy = 0.0;
            if (kFast || !single) {
                pair_force(psi2, psi1, psi0, k.negG, Fxd, Fyd);
                Fmx = Fxd;
                Fmy = kFast ? Fyd : Fyd - wall_adhesion_y(rB, psi1.c, k);
            } else {
                Fyd = wall_adhesion_y(rB, psi1.c, k);
            }
            const R rho = rhoPrv;
            R Fx = (R)Fxd + rho * drive_r + (rho - kr_.rho_v) * kr_.g_x;
            R Fy = (R)Fyd + (rho - kr_.rho_v) * kr_.g_y;
            const R rinv = rcp_r(rho);
            R ux = (jxPrv + (R)0.5 * Fx) * rinv;
            R uy = (jyPrv + (R)0.5 * Fy) * rinv;
            const bool resB = frame_rho && on_frame(rB);
            if (resB) ux = uy = 0;
            uxB = trix(ux);
            uyB = trix(uy);
            if (props) {  // lambda(rho(n)) of row kr-1, gas..liquid by the Eq. 5 fraction
                R fr = (rho - kr_.rho_g) * kr_.inv_drho;
                fr = fr < (R)0 ? (R)0 : (fr > (R)1 ? (R)1 : fr);
                lam1 = trix((R)k.lambda + (R)(k.lam_l - k.lambda) * fr);
            }
            if (kFast || (kr - 1 >= ya && kr - 1 < yb)) {
                // Eq. 8 theta term uses |F_m|^2 / psi^2 of the fluid-fluid force
                R th = 0;
                if ((kFast || !single) && psi1.c > 0.0)
                    th = (R)((Fmx * Fmx + Fmy * Fmy) * rcp_d<sizeof(S) == 4 ? 1 : 2>(psi1.c * psi1.c));
                // Eq. 5 with a clamped fraction
                R fr = (rho - kr_.rho_g) * kr_.inv_drho;
                fr = fr < (R)0 ? (R)0 : (fr > (R)1 ? (R)1 : fr);
                const R sv = rcp_r(kr_.tau_g + fr * kr_.dtau);
                R dn[9];
#pragma unroll
                for (int q = 0; q < 9; ++q) dn[q] = dPrv[q];
                collide<R>(dn, drPrv, rho, rinv, ux, uy, Fx, Fy, th, sv, cv);
                if (resB) {
                    const double dr = k.rho_frame - k.rho_ref;
#pragma unroll
                    for (int q = 0; q < 9; ++q)
                        dn[q] = (R)((q == 0 ? 4.0 / 9 : (q < 5 ? 1.0 / 9 : 1.0 / 36)) * dr);
                }
                // health of the node (state at level n): psi is 0 exactly
                // when Eq. 10 was clamped (a NaN argument too)
                auto count_health = [&]() {
                    health += psi1.c == 0.0 ? 1u : 0u;
                    if (!(__builtin_isfinite(rho) && __builtin_isfinite(tn1.c)))
                        health |= 0x80000000u;
                };
                if (!kHealthOnStore && own_lane) count_health();
                // The interior iteration of the plain FP32 build takes row kr+1
                // into its registers here, before the stores: the wait for the
                // loads then excludes these stores (one counter tracks both,
                // and a store block under a lane mask makes the compiler's
                // wait for the newest load a wait for everything issued).
                if (kEarlySettle && kFast) take_row();
                if (store_lane) {
                    if (kHealthOnStore) count_health();
                    const unsigned so = B.fout + (unsigned)rB.sr * rowb;
                    if (kMX) {
                        // rest population takes whatever keeps sum_i d_i equal to
                        // the pre-collision deviation density (FP64), as (hi, lo)
                        double rest = drdPrv;
#pragma unroll
                        for (int q = 1; q < 9; ++q) rest -= (double)(S)dn[q];
                        const float hi = (float)rest;
                        bstore((S)hi, rb, vx, so);
                        bstore((float)(rest - (double)hi), rb, vlo,
                               B.lo_out + (unsigned)rB.sr * rowb_lo);
                    } else {
                        bstore((S)dn[0], rb, vx, so);
                    }
#pragma unroll
                    for (int q = 1; q < 9; ++q) bstore((S)dn[q], rb, vx, q * P + so);
                }
            }
        } else {
            uxB = tri_const<R>(0);
            uyB = tri_const<R>(0);
            if (props) lam1 = tri_const<R>((R)k.lambda);  // solid nodes: gas values
        }
        ux1 = uxB;
        uy1 = uyB;

        if (kFast || !freezeT) {
            // ------------- stage C: div u, coefficients, h1 on row kr-2 ---
            const RowK rC = kFast ? row_interior(kr, 2) : row_info(kr - 2, g);
            Tri<R> t1;
            if (kFast || (rC.fluid && needC)) {
                const R dv = div_u<R>(ux3, ux2, ux1, uy3, uy2, uy1);
                R lam_c = cv.lambda, glx = 0, gly = 0, inv_cv = cv.inv_Cv;
                if (props) {
                    const R third = (R)1 / 3, twelfth = (R)1 / 12;
                    lam_c = lam2.c;
                    glx = lam2.d * third + (lam1.d + lam3.d) * twelfth;
                    gly = (lam1.c - lam3.c) * third + (lam1.a - lam3.a) * twelfth;
                    R fr = (rhoP2 - kr_.rho_g) * kr_.inv_drho;
                    fr = fr < (R)0 ? (R)0 : (fr > (R)1 ? (R)1 : fr);
                    inv_cv = rcp_r((R)(1.0 / k.inv_Cv) + (R)(k.cv_l - 1.0 / k.inv_Cv) * fr);
                }
                cf2 = heat_coef<R>(rhoP2, ux2.c, uy2.c, dv, T_ref + tn2.c, T_ref, cv, eos_cs,
                                   props, lam_c, glx, gly, inv_cv, kExt ? (R)k.alpha_max : (R)0);
                R h1 = heat_rhs<R>(tn3, tn2, tn1, cf2, T_ref);
                if (held(rC)) h1 = 0;
                acc2 = h1;
                t1 = trix(tn2.c + (R)0.5 * h1);
            } else {
                t1 = plate_t(kr - 2, t1b.c);
                acc2 = 0;
            }
            t1a = t1;
            // ------------- stage D: h2 on row kr-3 ------------------------
            const RowK rD = kFast ? row_interior(kr, 3) : row_info(kr - 3, g);
            Tri<R> t2;
            if (kFast || (rD.fluid && needD)) {
                R h2 = heat_rhs<R>(t1c, t1b, t1a, cf3, T_ref);
                if (held(rD)) h2 = 0;
                acc3 += (R)2 * h2;
                t2 = trix(tn3.c + (R)0.5 * h2);
            } else {
                t2 = plate_t(kr - 3, t2b.c);
            }
            t2a = t2;
            // ------------- stage E: h3 on row kr-4 ------------------------
            const RowK rE = kFast ? row_interior(kr, 4) : row_info(kr - 4, g);
            Tri<R> t3;
            if (kFast || (rE.fluid && needE)) {
                R h3 = heat_rhs<R>(t2c, t2b, t2a, cf4, T_ref);
                if (held(rE)) h3 = 0;
                acc4 += (R)2 * h3;
                t3 = trix(tn4 + h3);
            } else {
                t3 = plate_t(kr - 4, t3b.c);
            }
            t3a = t3;
            // ------------- stage F: h4 and T(n+1) on row kr-5 -------------
        }
        if (kAhead && !(kEarlySettle && kFast)) take_row();
        if (kFast || !freezeT) {
            const RowK rF = kFast ? row_interior(kr, 5) : row_info(kr - 5, g);
            if (kFast || (rF.fluid && kr - 5 >= ya && kr - 5 < yb)) {
                R h4 = heat_rhs<R>(t3c, t3b, t3a, cf5, T_ref);
                if (held(rF)) h4 = 0;
                const R tnew = tn5 + (acc5 + h4) * ((R)1 / 6);
                if (kOwnedTestAtT) {
                    // the owned-lane test is made here: the empty asm keeps
                    // the compiler from hoisting it out of the loop as a
                    // second live mask
                    int ln = lane;
                    asm volatile("" : "+v"(ln));
                    if (ln >= kHalo && ln < kHalo + own_w)
                        bstore((S)tnew, rb, vx, B.Tout + (unsigned)rF.sr * rowb);
                } else if (own_lane) {
                    bstore((S)tnew, rb, vx, B.Tout + (unsigned)rF.sr * rowb);
                }
            }
        }

        // ------------- shift the windows one row ---------------------------
        tn5 = tn4;
        tn4 = tn3.c;
        tn3 = tn2;
        tn2 = tn1;
        tn1 = tn0;
        psi2 = psi1;
        if (props) {
            lam3 = lam2;
            lam2 = lam1;
        }
        psi1 = psi0;
        ux3 = ux2;
        ux2 = ux1;
        uy3 = uy2;
        uy2 = uy1;
        cf5 = cf4;
        cf4 = cf3;
        cf3 = cf2;
        acc5 = acc4;
        acc4 = acc3;
        acc3 = acc2;
        t1c = t1b;
        t1b = t1a;
        t2c = t2b;
        t2b = t2a;
        t3c = t3b;
        t3b = t3a;
        rhoP2 = rhoPrv;
        rhoPrv = rhoCur;
        drPrv = drCur;
        jxPrv = jxCur;
        jyPrv = jyCur;
        drdPrv = drdCur;
#pragma unroll
        for (int q = 0; q < 9; ++q) dPrv[q] = dCur[q];

    };
    // interior iterations: kr - 5 .. kr + 1 inside the segment's owned rows
    // and the stages' reach, all rows at least two rows off the plates
    const bool fast_ok = !kExt && !freezeT && !single && !g.periodic_y;
    const int fast_lo = max(ya + kHalo, 6), fast_hi = min(yb, g.Ny - 4);
    auto step_row = [&](const int kr) {
        if constexpr (!kExt) {
            if (fast_ok && kr >= fast_lo && kr <= fast_hi) {
                row_iteration(kr, std::true_type{});
                return;
            }
        }
        row_iteration(kr, std::false_type{});
    };
    for (int kr = ya - kHalo; kr < kr_end; kr += 6) {
        step_row(kr);
        step_row(kr + 1);
        step_row(kr + 2);
        step_row(kr + 3);
        step_row(kr + 4);
        step_row(kr + 5);
    }
    flush_health(B.stat, health);
}

// wave index inside the block, as a wave-uniform value
__device__ __forceinline__ int wave_in_block() {
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// The FP64 build has its own kernel: it needs about 256 registers.
// Register budgets: three waves per SIMD for the FP32 deviation build (168
// VGPRs), two for the FP64 build (256) and for the mass-exact build, whose
// FP64 density and split rest population need about 178 (held to 168 it
// spills some 9 registers to scratch inside the row loop, which costs more
// than the third wave gains); the interior path would otherwise take a few
// more registers than that and lose a resident wave.
template <class S, bool kMX, bool kExt>
__global__ __launch_bounds__(kLanes* kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(kMX ? 2 : 3)))
void step_kernel(Grid g, Phys k, Bufs<S> B,
                                                                        long long n) {
    const int unit = unit_of_block(g.n_blocks_pad) * kWavesPerBlock + wave_in_block();
    if (unit >= g.n_units) return;  // whole waves only
    const double rin = (kExt && g.open_x) ? inlet_density(k, n) : 0.0;
    step_unit<S, kMX, kExt>(g, k, B, drive_at(k, n), rin, unit);
}

template <bool kExt>
__global__ __launch_bounds__(kLanes* kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(2)))
void step_kernel_f64(Grid g, Phys k,
                                                                        Bufs<double> B,
                                                                        long long n) {
    const int unit = unit_of_block(g.n_blocks_pad) * kWavesPerBlock + wave_in_block();
    if (unit >= g.n_units) return;
    const double rin = (kExt && g.open_x) ? inlet_density(k, n) : 0.0;
    step_unit<double, false, kExt>(g, k, B, drive_at(k, n), rin, unit);
}

// Step i of a chunk over a batch of channels.  The slot of a unit is found by
// a binary search over the slots' first units (wave-uniform).
template <bool kExt>
__global__ __launch_bounds__(kLanes* kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(3)))
void step_batched_kernel(
    const Slot* __restrict__ slots, int n_slots, int total_units, int nblocks_pad, int step_i) {
    const int unit = unit_of_block(nblocks_pad) * kWavesPerBlock + wave_in_block();
    if (unit >= total_units) return;
    int lo = 0, hi = n_slots - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (slots[mid].unit_begin <= unit) lo = mid; else hi = mid - 1;
    }
    const Slot& sl = slots[lo];
    if (step_i >= sl.steps_left) return;
    // local copies: the buffer stores of the step may alias the table as far
    // as the compiler can tell, which would force reloads inside the loop
    const Grid g = sl.g;
    const Phys k = sl.k;
    Bufs<float> B;
    B.base = sl.mem;
    B.span = sl.span;
    const int a = (sl.cur_f + step_i) & 1;
    B.fin = sl.off_f[a];
    B.fout = sl.off_f[a ^ 1];
    B.lo_in = B.lo_out = 0;
    B.stat = sl.stat;
    if (sl.k.flags & kFreezeT) {
        B.Tin = B.Tout = sl.off_T[sl.cur_T];
    } else {
        const int t = (sl.cur_T + step_i) & 1;
        B.Tin = sl.off_T[t];
        B.Tout = sl.off_T[t ^ 1];
    }
    const double rin = (kExt && g.open_x) ? inlet_density(k, sl.n0 + step_i) : 0.0;
    step_unit<float, false, kExt>(g, k, B, drive_at(k, sl.n0 + step_i), rin,
                                  unit - sl.unit_begin);
}

// ---- moments: two passes over all nodes ------------------------------------
// a node of a FRAME_RHO reservoir (y counts the plate rows)
__device__ __forceinline__ bool reservoir_node(const Grid& g, int cx, int y) {
    return g.frame_rho &&
           (cx == 0 || cx == g.Nx - 1 || (g.periodic_y && (y == 0 || y == g.Ny - 1)));
}

// The read-out's arithmetic per node, shared by the two-pass read-out and
// the one-pass reduction, so that both see bitwise the same node values.
struct NodeState {
    double rho, psi, jx, jy, T;  // rho = 0 and j = 0 on plate rows
    bool fluid;
};

// rho, psi, j and T of node (cx, y) (y counts the plate rows) at time level
// n_t from the stored post-collision state.
template <class S, bool kMX>
__device__ __forceinline__ NodeState node_state(const Grid& g, const Phys& k,
                                                const S* __restrict__ f,
                                                const float* __restrict__ f0lo,
                                                const S* __restrict__ T, int cx, int y,
                                                long long n_t) {
    NodeState o;
    const RowK r = row_info(y, g);
    o.fluid = r.fluid;
    if (!r.fluid) {
        o.psi = k.psi_wall_eff;
        o.jx = o.jy = 0.0;
        o.rho = 0.0;
        o.T = k.T_ref + (k.wall_ramp ? k.dT_wall + (k.dT_w_end - k.dT_wall) * (double)cx /
                                                       (double)(g.Nx - 1)
                         : ((k.flags & kTopMixed) && y == 0) ? k.dT_w_bot
                                                             : k.dT_wall);
        return o;
    }
    const unsigned x = (unsigned)cx;
    const unsigned xm = (unsigned)(cx == 0 ? g.Nx - 1 : cx - 1);
    const unsigned xp = (unsigned)(cx == g.Nx - 1 ? 0 : cx + 1);
    S d[9];
    pull_row<S>(f, g, r, x, xm, xp, d);
    if (g.open_x && (cx == 0 || cx == g.Nx - 1)) {
        using R = typename RealOf<S>::T;
        R dr_[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) dr_[q] = (R)d[q];
        zou_he<R>(dr_, cx == 0, cx == g.Nx - 1, cx == 0 ? inlet_density(k, n_t) : 0.0, k,
                  r.bb_lo || r.bb_hi);
#pragma unroll
        for (int q = 0; q < 9; ++q) d[q] = (S)dr_[q];
    }
    double dr = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) dr += (double)d[q];
    if (kMX) dr += (double)f0lo[(unsigned)r.sr * (unsigned)g.pitch + x];
    const bool res = reservoir_node(g, cx, y);
    if (res) dr = k.rho_frame - k.rho_ref;
    o.rho = k.rho_ref + dr;
    o.T = k.T_ref + (double)T[(unsigned)r.sr * (unsigned)g.pitch + x];
    bool clamped;
    o.psi = psi_eos<sizeof(S) == 4>(o.rho, o.T, k, clamped);
    o.jx = ((double)d[1] - (double)d[3]) + ((double)d[5] - (double)d[6]) +
           ((double)d[8] - (double)d[7]);
    o.jy = ((double)d[2] - (double)d[4]) + ((double)d[5] + (double)d[6]) -
           ((double)d[7] + (double)d[8]);
    if (res) o.jx = o.jy = 0.0;
    return o;
}

// u of a fluid node (Eq. 13) from its rho and j and the psi of the rows
// below (pS), at (pC) and above (pN) it, each as centre / x-sum / x-difference.
__device__ __forceinline__ void node_velocity(const Grid& g, const Phys& k, int cx, int y,
                                              const Tri<double>& pS, const Tri<double>& pC,
                                              const Tri<double>& pN, double rho, double jx,
                                              double jy, long long n_t, double& ux,
                                              double& uy) {
    const RowK r = row_info(y, g);
    double Fx = 0.0, Fy = 0.0;
    if (!(k.flags & kSinglePhase))
        pair_force(pS, pC, pN, k.negG, Fx, Fy);
    else
        Fy = wall_adhesion_y(r, pC.c, k);
    Fx += rho * drive_at(k, n_t) + (rho - k.rho_v) * k.g_x;
    Fy += (rho - k.rho_v) * k.g_y;
    ux = (jx + 0.5 * Fx) / rho;
    uy = (jy + 0.5 * Fy) / rho;
    if (reservoir_node(g, cx, y)) ux = uy = 0.0;
}

// the x-neighbours the read-out uses: periodic, or past an open end the end
// column itself
__device__ __forceinline__ int read_xm(const Grid& g, int cx) {
    return cx == 0 ? (g.open_x ? 0 : g.Nx - 1) : cx - 1;
}
__device__ __forceinline__ int read_xp(const Grid& g, int cx) {
    return cx == g.Nx - 1 ? (g.open_x ? cx : 0) : cx + 1;
}

// pass 1: rho, psi, j (and T) per node into scratch; pass 2: forces and u.
template <class S, bool kMX>
__global__ __launch_bounds__(256) void moments_pass1(Grid g, Phys k, const S* __restrict__ f,
                                                     const float* __restrict__ f0lo,
                                                     const S* __restrict__ T,
                                                     double* __restrict__ work,
                                                     double* __restrict__ rho_out,
                                                     double* __restrict__ T_out, long long n_t,
                                                     unsigned long long* __restrict__ n_bad) {
    const int n = g.Nx * g.Ny;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int y = i / g.Nx, cx = i - y * g.Nx;
    const NodeState o = node_state<S, kMX>(g, k, f, f0lo, T, cx, y, n_t);
    work[i] = o.psi;
    work[n + i] = o.jx;
    work[2 * n + i] = o.jy;
    rho_out[i] = o.rho;
    T_out[i] = o.T;
    if (o.fluid && !(__builtin_isfinite(o.rho) && __builtin_isfinite(o.T))) atomicAdd(n_bad, 1ull);
}

__global__ __launch_bounds__(256) void moments_pass2(Grid g, Phys k,
                                                     const double* __restrict__ work,
                                                     const double* __restrict__ rho_in,
                                                     double* __restrict__ ux_out,
                                                     double* __restrict__ uy_out, long long n_t) {
    const int n = g.Nx * g.Ny;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int y = i / g.Nx, cx = i - y * g.Nx;
    const RowK r = row_info(y, g);
    if (!r.fluid) {
        ux_out[i] = uy_out[i] = 0.0;
        return;
    }
    const double* psi = work;
    const double* jx = work + n;
    const double* jy = work + 2 * n;
    const int xm = read_xm(g, cx), xp = read_xp(g, cx);
    int ys = y - 1, yn = y + 1;
    if (g.periodic_y) {
        if (ys < 0) ys += g.Ny;
        if (yn >= g.Ny) yn -= g.Ny;
    }
    auto row3 = [&](int yy) {
        const double m = psi[yy * g.Nx + xm], p = psi[yy * g.Nx + xp];
        Tri<double> t;
        t.c = psi[yy * g.Nx + cx];
        t.a = p + m;
        t.d = p - m;
        return t;
    };
    double ux, uy;
    node_velocity(g, k, cx, y, row3(ys), row3(y), row3(yn), rho_in[i], jx[i], jy[i], n_t, ux,
                  uy);
    ux_out[i] = ux;
    uy_out[i] = uy;
}

// ---- initial state ----------------------------------------------------------
// Buffers hold post-collision values, so the start state is the field that
// the first pull turns into f_i(x, 0) = w_i rho0(x): d*_i(z) = w_i (rho0(z + e_i)
// - rho_ref), or w_i (rho0(z) - rho_ref) where z + e_i is a plate.
template <class S, bool kMX>
__global__ __launch_bounds__(256) void init_kernel(Grid g, Phys k, const double* __restrict__ rho0,
                                                   S* __restrict__ f, float* __restrict__ f0lo,
                                                   S* __restrict__ T) {
    const int n = g.rows * g.Nx;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int sr = i / g.Nx, cx = i - sr * g.Nx;
    const int y = sr + g.y_first;
    const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                         1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    const unsigned o = (unsigned)sr * (unsigned)g.pitch + (unsigned)cx;
    for (int q = 0; q < 9; ++q) {
        int tx = cx + ex[q];
        tx = tx < 0 ? tx + g.Nx : (tx >= g.Nx ? tx - g.Nx : tx);
        int ty = y + ey[q];
        bool solid = false;
        if (g.periodic_y) {
            ty = ty < 0 ? ty + g.Ny : (ty >= g.Ny ? ty - g.Ny : ty);
        } else {
            solid = (ty == 0 || ty == g.Ny - 1);
        }
        const double r = solid ? rho0[y * g.Nx + cx] : rho0[ty * g.Nx + tx];
        const double v = w[q] * (r - k.rho_ref);
        if (kMX && q == 0) {
            const float hi = (float)v;
            f[o] = (S)hi;
            f0lo[o] = (float)(v - (double)hi);
        } else {
            f[q * g.plane + o] = (S)v;
        }
    }
    // T = T_0 = T_ref, T_w on a held frame node, T_in on an open inlet,
    // T_out on a held open outlet
    const bool held = g.frame_t && (cx == 0 || cx == g.Nx - 1 ||
                                    (g.periodic_y && (y == 0 || y == g.Ny - 1)));
    T[o] = (g.open_x && cx == 0)
               ? (S)k.dT_in
               : ((g.open_x && k.hold_out && cx == g.Nx - 1) ? (S)k.dT_out
                                                             : (held ? (S)k.dT_wall : (S)0));
}

// ---- deterministic FP64 reduction ------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(256) void reduce_pass1(const double* __restrict__ rho,
                                                    const double* __restrict__ ux,
                                                    const double* __restrict__ uy,
                                                    const double* __restrict__ T, int n,
                                                    double Cv, double* __restrict__ partials) {
    double s[5] = {0, 0, 0, 0, 0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double r = rho[i], a = ux[i], b = uy[i], t = T[i];
        if (!(isfinite(r) && isfinite(a) && isfinite(b) && isfinite(t))) {
            s[4] += 1.0;
            continue;
        }
        s[0] += r;
        s[1] += r * a;
        s[2] += r * b;
        s[3] += r * Cv * t;
    }
    __shared__ double red[4][5];
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const double t = wave_sum(s[q]);
        if (ln == 0) red[wv][q] = t;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        const int q = threadIdx.x;
        partials[blockIdx.x * 5 + q] = ((red[0][q] + red[1][q]) + (red[2][q] + red[3][q]));
    }
}

__global__ __launch_bounds__(64) void reduce_pass2(const double* __restrict__ partials, int nb,
                                                   double* __restrict__ out) {
    if (threadIdx.x < 5) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += partials[b * 5 + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// ---- one-pass reduction from the state (allocation-free entry point) ------
// A block takes tiles of 64 columns x 4 rows in a fixed order (tile
// blockIdx.x, then every gridDim.x-th).  For a tile it evaluates psi on the
// tile and its one-node ring into LDS (66 x 6 nodes, the ring recomputed),
// then every node of the tile its u from its own state and the psi of its
// neighbours, and adds rho, rho u_x, rho u_y, rho C_v T and the non-finite
// count in FP64.  Block totals go to part[5 * blockIdx.x + q] (every entry
// written, nothing needs clearing); reduce_pass2 sums them in block order.
constexpr int kTileW = 64, kTileH = 4;
constexpr int kRingW = kTileW + 2, kRingH = kTileH + 2;

template <class S, bool kMX>
__global__ __launch_bounds__(256) void reduce_state_kernel(Grid g, Phys k,
                                                           const S* __restrict__ f,
                                                           const float* __restrict__ f0lo,
                                                           const S* __restrict__ T, double Cv,
                                                           long long n_t,
                                                           double* __restrict__ part) {
    __shared__ double psi_t[kRingH][kRingW];
    const int tiles_x = (g.Nx + kTileW - 1) / kTileW;
    const int tiles = tiles_x * ((g.Ny + kTileH - 1) / kTileH);
    const int tx = threadIdx.x & (kTileW - 1), ty = threadIdx.x >> 6;
    double s[5] = {0, 0, 0, 0, 0};
    for (int t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int x0 = (t % tiles_x) * kTileW, y0 = (t / tiles_x) * kTileH;
        __syncthreads();  // the previous tile's readers are done
        for (int e = threadIdx.x; e < kRingW * kRingH; e += blockDim.x) {
            const int ex = e % kRingW, ey = e / kRingW;
            // ring columns map as the read-out's neighbours do (periodic or
            // the end column past an open end); entries no node reads are
            // left unset
            int cx = x0 - 1 + ex;
            if (cx < 0) cx = read_xm(g, 0);
            else if (cx >= g.Nx) cx = cx == g.Nx ? read_xp(g, g.Nx - 1) : -1;
            int y = y0 - 1 + ey;
            if (g.periodic_y) y = y < 0 ? y + g.Ny : (y >= g.Ny ? y - g.Ny : y);
            else if (y < 0 || y >= g.Ny) y = -1;
            if (cx >= 0 && y >= 0 && y < g.Ny)
                psi_t[ey][ex] = node_state<S, kMX>(g, k, f, f0lo, T, cx, y, n_t).psi;
        }
        __syncthreads();
        const int cx = x0 + tx, y = y0 + ty;
        if (cx < g.Nx && y < g.Ny) {
            const NodeState o = node_state<S, kMX>(g, k, f, f0lo, T, cx, y, n_t);
            if (o.fluid) {
                auto row3 = [&](int ey) {
                    const double m = psi_t[ey][tx], p = psi_t[ey][tx + 2];
                    Tri<double> r;
                    r.c = psi_t[ey][tx + 1];
                    r.a = p + m;
                    r.d = p - m;
                    return r;
                };
                double ux, uy;
                node_velocity(g, k, cx, y, row3(ty), row3(ty + 1), row3(ty + 2), o.rho, o.jx,
                              o.jy, n_t, ux, uy);
                if (!(isfinite(o.rho) && isfinite(ux) && isfinite(uy) && isfinite(o.T))) {
                    s[4] += 1.0;
                } else {
                    s[0] += o.rho;
                    s[1] += o.rho * ux;
                    s[2] += o.rho * uy;
                    s[3] += o.rho * Cv * o.T;
                }
            }
        }
    }
    __shared__ double red[4][5];
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const double v = wave_sum(s[q]);
        if (ln == 0) red[wv][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        const int q = threadIdx.x;
        part[blockIdx.x * 5 + q] = ((red[0][q] + red[1][q]) + (red[2][q] + red[3][q]));
    }
}

inline int blocks_for(int n, int bs) { return (n + bs - 1) / bs; }

// ---- plain copy for the bandwidth probe -----------------------------------
// One 16-byte vector per thread, streaming (non-temporal) loads and stores:
// the fastest of the plain copy forms measured on MI355X (grid-stride loops
// with 2k-128k blocks, unrolled by 1 and 4, with and without the
// non-temporal hint), so the probe is a fair ceiling for the step kernel.
typedef float f32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void copy_kernel(const f32x4* __restrict__ src,
                                                   f32x4* __restrict__ dst, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(&src[i]), &dst[i]);
}

}  // namespace

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 16;
    const size_t blocks = (n + 255) / 256;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const f32x4*>(src), static_cast<f32x4*>(dst), n);
    return hipGetLastError();
}

bool needs_ext(const Grid& g, const Phys& k) {
    return g.frame_t || g.frame_rho || g.open_x || k.wall_ramp || k.alpha_max > 0.0 ||
           (k.flags & (kEosCS | kPhaseProps | kTopMixed));
}

template <class S, bool kMX>
static hipError_t step_impl(const Grid& g, const Phys& k, const Bufs<S>& b, int64_t n,
                            hipStream_t s) {
    if (g.n_units <= 0) return hipSuccess;
    if (needs_ext(g, k))
        hipLaunchKernelGGL((step_kernel<S, kMX, true>), dim3(g.n_blocks_pad),
                           dim3(kLanes * kWavesPerBlock), 0, s, g, k, b, (long long)n);
    else
        hipLaunchKernelGGL((step_kernel<S, kMX, false>), dim3(g.n_blocks_pad),
                           dim3(kLanes * kWavesPerBlock), 0, s, g, k, b, (long long)n);
    return hipGetLastError();
}

hipError_t launch_step_f32(const Grid& g, const Phys& k, const Bufs<float>& b, bool mass_exact,
                           int64_t n, hipStream_t s) {
    return mass_exact ? step_impl<float, true>(g, k, b, n, s)
                      : step_impl<float, false>(g, k, b, n, s);
}
hipError_t launch_step_f64(const Grid& g, const Phys& k, const Bufs<double>& b, int64_t n,
                           hipStream_t s) {
    if (g.n_units <= 0) return hipSuccess;
    if (needs_ext(g, k))
        hipLaunchKernelGGL(step_kernel_f64<true>, dim3(g.n_blocks_pad),
                           dim3(kLanes * kWavesPerBlock), 0, s, g, k, b, (long long)n);
    else
        hipLaunchKernelGGL(step_kernel_f64<false>, dim3(g.n_blocks_pad),
                           dim3(kLanes * kWavesPerBlock), 0, s, g, k, b, (long long)n);
    return hipGetLastError();
}

hipError_t launch_step_batched(const Slot* slots, int n_slots, int total_units, int step_i,
                               bool ext, hipStream_t s) {
    if (total_units <= 0 || n_slots <= 0) return hipSuccess;
    const int nb = (total_units + kWavesPerBlock - 1) / kWavesPerBlock;
    const int nbp = (nb + 7) / 8 * 8;
    if (ext)
        hipLaunchKernelGGL(step_batched_kernel<true>, dim3(nbp), dim3(kLanes * kWavesPerBlock), 0,
                           s, slots, n_slots, total_units, nbp, step_i);
    else
        hipLaunchKernelGGL(step_batched_kernel<false>, dim3(nbp), dim3(kLanes * kWavesPerBlock), 0,
                           s, slots, n_slots, total_units, nbp, step_i);
    return hipGetLastError();
}

template <class S, bool kMX>
static hipError_t moments_impl(const Grid& g, const Phys& k, const S* f, const float* f0lo,
                               const S* T, double* work, double* rho, double* ux, double* uy,
                               double* Tout, int64_t n_t, unsigned long long* n_bad,
                               hipStream_t s) {
    const int n = g.Nx * g.Ny;
    hipLaunchKernelGGL((moments_pass1<S, kMX>), dim3(blocks_for(n, 256)), dim3(256), 0, s, g, k,
                       f, f0lo, T, work, rho, Tout, (long long)n_t, n_bad);
    hipLaunchKernelGGL(moments_pass2, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, k,
                       (const double*)work, (const double*)rho, ux, uy, (long long)n_t);
    return hipGetLastError();
}

hipError_t launch_moments_f32(const Grid& g, const Phys& k, const float* f, const float* f0lo,
                              const float* T, double* work, double* rho, double* ux,
                              double* uy, double* Tout, int64_t n, unsigned long long* n_bad,
                              hipStream_t s) {
    if (f0lo)
        return moments_impl<float, true>(g, k, f, f0lo, T, work, rho, ux, uy, Tout, n, n_bad, s);
    return moments_impl<float, false>(g, k, f, nullptr, T, work, rho, ux, uy, Tout, n, n_bad, s);
}
hipError_t launch_moments_f64(const Grid& g, const Phys& k, const double* f, const double* T,
                              double* work, double* rho, double* ux, double* uy,
                              double* Tout, int64_t n, unsigned long long* n_bad, hipStream_t s) {
    return moments_impl<double, false>(g, k, f, nullptr, T, work, rho, ux, uy, Tout, n, n_bad,
                                       s);
}

hipError_t launch_init_f32(const Grid& g, const Phys& k, const double* rho0, float* f,
                           float* f0lo, float* T, hipStream_t s) {
    const int n = g.rows * g.Nx;
    if (f0lo)
        hipLaunchKernelGGL((init_kernel<float, true>), dim3(blocks_for(n, 256)), dim3(256), 0, s,
                           g, k, rho0, f, f0lo, T);
    else
        hipLaunchKernelGGL((init_kernel<float, false>), dim3(blocks_for(n, 256)), dim3(256), 0, s,
                           g, k, rho0, f, f0lo, T);
    return hipGetLastError();
}
hipError_t launch_init_f64(const Grid& g, const Phys& k, const double* rho0, double* f,
                           double* T, hipStream_t s) {
    const int n = g.rows * g.Nx;
    hipLaunchKernelGGL((init_kernel<double, false>), dim3(blocks_for(n, 256)), dim3(256), 0, s,
                       g, k, rho0, f, (float*)nullptr, T);
    return hipGetLastError();
}

// ---- allocation-free reduction: file-scope scratch -------------------------
// Block partials of reduce_state_kernel for callers that cannot allocate:
// kStaticReduceBlocks x 5 doubles (40 KiB) per GPU, held until the process
// ends.  Host code never uses the array's name as an address: each device's
// copy is resolved once with hipGetSymbolAddress (that device current) and
// the resolved pointer is passed to the kernels.
static __device__ __align__(256) double scratch[kStaticReduceBlocks * 5];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// this device's copy of `scratch` (resolved on its first use)
hipError_t scratch_on_current_device(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<double*>(g_scratch_ptr[dev]);
    return hipSuccess;
}

template <class S, bool kMX>
hipError_t reduce_state_impl(const Grid& g, const Phys& k, const S* f, const float* f0lo,
                             const S* T, double Cv, int64_t n_t, double* out_dev,
                             hipStream_t s) {
    double* part = nullptr;
    hipError_t e = scratch_on_current_device(&part);
    if (e != hipSuccess) return e;
    const long long tiles = (long long)((g.Nx + kTileW - 1) / kTileW) *
                            ((g.Ny + kTileH - 1) / kTileH);
    const int nb = (int)std::min<long long>(tiles, kStaticReduceBlocks);
    hipLaunchKernelGGL((reduce_state_kernel<S, kMX>), dim3(nb), dim3(kTileW * kTileH), 0, s, g,
                       k, f, f0lo, T, Cv, (long long)n_t, part);
    hipLaunchKernelGGL(reduce_pass2, dim3(1), dim3(64), 0, s, (const double*)part, nb, out_dev);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_reduce_state_f32(const Grid& g, const Phys& k, const float* f,
                                   const float* f0lo, const float* T, double Cv, int64_t n_t,
                                   double* out_dev, hipStream_t s) {
    if (f0lo) return reduce_state_impl<float, true>(g, k, f, f0lo, T, Cv, n_t, out_dev, s);
    return reduce_state_impl<float, false>(g, k, f, nullptr, T, Cv, n_t, out_dev, s);
}
hipError_t launch_reduce_state_f64(const Grid& g, const Phys& k, const double* f, const double* T,
                                   double Cv, int64_t n_t, double* out_dev, hipStream_t s) {
    return reduce_state_impl<double, false>(g, k, f, nullptr, T, Cv, n_t, out_dev, s);
}

hipError_t launch_reduce(const double* rho, const double* ux, const double* uy, const double* T,
                         int n, double Cv, double* partials, double* out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_pass1, dim3(kReduceBlocks), dim3(256), 0, s, rho, ux, uy, T, n, Cv,
                       partials);
    hipLaunchKernelGGL(reduce_pass2, dim3(1), dim3(64), 0, s, (const double*)partials,
                       kReduceBlocks, out);
    return hipGetLastError();
}

}  // namespace lbmk
