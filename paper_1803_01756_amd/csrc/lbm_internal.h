// Internal interface between the C-ABI runtime (lbm_runtime.cpp) and the
// HIP kernels (lbm_kernels.hip).  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lbmk {

// Owned columns per wave-strip: 64 lanes minus a 5-column halo on each side
// (psi needs rho one column out, u needs psi one further, and each of the four
// RK4 stages widens the temperature stencil by one more column).
constexpr int kLanes = 64;
constexpr int kHalo = 5;
constexpr int kOwned = kLanes - 2 * kHalo;

// Constants that enter arithmetic done in the storage precision R, given in
// R on the host so that the kernels never convert them per use.
template <class R>
struct PhysR {
    R s_rho, s_e, s_z, s_j, s_q, c_e, c_z;
    R b, rkA, rkB1, rkB2, inv_Cv, lambda;
    R T_ref, dT_wall, rho_ref, rho_v, g_x, g_y;
    R rho_g, inv_drho, tau_g, dtau;
};

// Uniform physical constants, resolved on the host in FP64.  The kernels
// read them from the kernel-argument segment (scalar registers).
struct Phys {
    double rho_ref, T_ref, dT_wall;     // storage references; T_w - T_ref
    double a, b, R, kappa, inv_Tc;      // Eq. 11
    double inv_G, negG;                 // Eq. 10 (1/G) and Eq. 9 (-G)
    double psi_wall_eff;                // psi_w G_w / G: solid-row potential
    double Gw_psiw;                     // G_w psi_w (Eq. 14 on the wall rows)
    double c_e, c_z;                    // 12 theta / (tau_e - 1/2), same for zeta
    double s_rho, s_e, s_z, s_j, s_q;   // Eq. 3 rates
    double tau_g, dtau, rho_g, inv_drho;// Eq. 5 (inv_drho = 0: constant tau)
    double inv_Cv, lambda;              // Eq. 16
    double g_osc, period;               // drive g_osc sin(2 pi n / period) along +x
    double g_x, g_y, rho_v;             // Eq. 15
    double rho_frame;                   // reservoir density of a frame
    double p0, p_amp, p_period;         // open ends: inlet pressure p0 (1 + p_amp sin(...))
    double T_in_eos;                    // temperature of the boundary EOS pressures
    double rho_sp;                      // vapour spinodal density at T_in_eos (bracket)
    double dT_in;                       // inlet temperature - T_ref
    double dT_out;                      // held outlet temperature - T_ref (hold_out)
    int hold_out;                       // the outlet column holds its temperature
    double alpha_max;                   // > 0: cap of lambda / (rho C_v) in the conduction term
    double dT_w_end;                    // plate temperature at x = Nx-1 - T_ref
    int wall_ramp;                      // plate temperature linear in x
    double lam_l, cv_l;                 // liquid conductivity and heat capacity
    double dT_w_bot;                    // bottom plate temperature - T_ref (TOP_MIXED)
    int cold_x0, cold_x1;               // cold columns of the top plate (TOP_MIXED)
    double rkA, rkB1, rkB2;             // R, a k (1+k)/sqrt(Tc), a k^2 / Tc
    uint32_t flags;                     // LBM_FREEZE_T | LBM_SINGLE_PHASE | LBM_PERIODIC_Y
    uint32_t pad_;
    PhysR<float> rf;                    // the same constants in FP32 and FP64
    PhysR<double> rd;
};

struct Grid {
    int Nx, Ny;        // nodes incl. plate rows
    int pitch;         // elements per stored row (multiple of 64)
    int rows;          // stored (fluid) rows
    int y_first;       // y of stored row 0 (1 with plates, 0 periodic)
    int periodic_y;
    int frame_t;       // T held at T_w on the frame: outermost columns (and rows if periodic_y)
    int frame_rho;     // the frame is a reservoir at rest with density rho_frame
    int open_x;        // Zou-He pressure inlet at x = 0, outlet at x = Nx-1
    int n_strips, n_segs, seg_rows, n_units, n_blocks_pad;
    unsigned plane;    // rows * pitch
};

// Every buffer a step touches lies in one device allocation; the kernel
// reaches them all through one buffer resource on `base`, by byte offsets.
template <class S>
struct Bufs {
    const char* base;         // the allocation
    unsigned span;            // bytes from base to the end of the last buffer
    unsigned fin, fout;       // population buffers: 9 planes of S
    unsigned lo_in, lo_out;   // mass-exact low parts of the rest population (float)
    unsigned Tin, Tout;       // temperature planes (Tout unused when T is frozen)
    // health counters, added to by every step: [0] owned nodes whose state
    // at the step's time level holds a non-finite rho or T, [1] owned nodes
    // whose Eq. 10 argument was clamped (psi = 0)
    unsigned long long* stat;
};

constexpr int kWavesPerBlock = 4;

// One fused time step n -> n+1 (pull-stream + bounce-back, psi, forces, u,
// MRT collision, RK4 temperature) over all units of the grid.
hipError_t launch_step_f32(const Grid& g, const Phys& k, const Bufs<float>& b, bool mass_exact,
                           int64_t n, hipStream_t s);
hipError_t launch_step_f64(const Grid& g, const Phys& k, const Bufs<double>& b, int64_t n,
                           hipStream_t s);

// One channel of a batch (FP32 deviation storage).  The table of slots is
// constant during a chunk of steps; step i of the chunk reads buffer
// (cur + i) & 1 and writes the other, at time level n0 + i, and a slot takes
// part only while i < steps_left.
struct Slot {
    Grid g;
    Phys k;
    const char* mem;          // the slot's allocation
    unsigned span;            // bytes of it the step touches
    unsigned off_f[2];        // byte offsets of the population buffers
    unsigned off_T[2];        // and of the temperature planes
    int64_t n0;
    int cur_f, cur_T;
    int steps_left;
    int unit_begin;  // first unit of this slot in the batch numbering
    unsigned long long* stat;  // the slot's health counters (see Bufs::stat)
};

// Step i of a chunk over every slot of the table (slots sorted by
// unit_begin, total_units = sum of their units).
// ext: some slot uses an optional feature (frames, Carnahan-Starling EOS,
// open ends, plate temperature ramp, phase-dependent properties, Sec. 3.2
// plates), so the batch runs the kernel build that has them
hipError_t launch_step_batched(const Slot* slots, int n_slots, int total_units, int step_i, bool ext,
                               hipStream_t s);

// rho, u (half force) and T at the current time level into device arrays of
// Nx*Ny doubles; work holds 3*Nx*Ny doubles; *n_bad is incremented for
// every fluid node whose rho or T is not finite.
hipError_t launch_moments_f32(const Grid& g, const Phys& k, const float* f, const float* f0lo,
                              const float* T, double* work, double* rho, double* ux,
                              double* uy, double* Tout, int64_t n, unsigned long long* n_bad,
                              hipStream_t s);
hipError_t launch_moments_f64(const Grid& g, const Phys& k, const double* f, const double* T,
                              double* work, double* rho, double* ux, double* uy,
                              double* Tout, int64_t n, unsigned long long* n_bad, hipStream_t s);

// Rest-equilibrium start from a device density field rho0 (Nx*Ny doubles).
hipError_t launch_init_f32(const Grid& g, const Phys& k, const double* rho0, float* f,
                           float* f0lo, float* T, hipStream_t s);
hipError_t launch_init_f64(const Grid& g, const Phys& k, const double* rho0, double* f,
                           double* T, hipStream_t s);

// Deterministic FP64 reduction of the moment arrays: out[5] = {sum rho,
// sum rho ux, sum rho uy, sum rho Cv T, non-finite count}.  partials holds
// kReduceBlocks*5 doubles.
constexpr int kReduceBlocks = 256;
hipError_t launch_reduce(const double* rho, const double* ux, const double* uy,
                         const double* T, int n, double Cv, double* partials, double* out,
                         hipStream_t s);

// The totals of launch_reduce (out_dev[5], device memory) computed in one
// pass from the stored state at time level n_t, with the block partials in
// the library's file-scope scratch array (kStaticReduceBlocks blocks at
// most; no allocation, no clearing): the allocation-free reduction.  Calls
// that overlap on one device share that scratch and race.
constexpr int kStaticReduceBlocks = 1024;
hipError_t launch_reduce_state_f32(const Grid& g, const Phys& k, const float* f,
                                   const float* f0lo, const float* T, double Cv, int64_t n_t,
                                   double* out_dev, hipStream_t s);
hipError_t launch_reduce_state_f64(const Grid& g, const Phys& k, const double* f, const double* T,
                                   double Cv, int64_t n_t, double* out_dev, hipStream_t s);

// Plain device copy of bytes (a multiple of 16) for the bandwidth probe.
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);

}  // namespace lbmk
