// Host helpers shared by the single-channel runtime and the slot pool.
// Internal; not part of the C-ABI.
#pragma once

#include <cstddef>

#include "lbm.h"
#include "lbm_internal.h"

namespace lbmhost {

constexpr int kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Elements added to the population plane stride beyond pitch x rows (a
// multiple of 64, so rows keep their 256-byte alignment).  When pitch x rows
// is a multiple of a large power of two (8192 x 510 FP32 values are
// 255 x 64 KiB) the nine planes of one row start at addresses that agree in
// all their low bits and their loads and stores pile onto the same HBM
// channels; skewing each plane by 3.25 KiB (FP32) spreads them.
constexpr size_t kPlaneSkew = 832;

// Device memory layout of one channel: two population buffers
// [9][rows][pitch] with a plane stride of pitch x rows + kPlaneSkew,
// optional mass-exact low planes, two temperature planes, then the moment
// arrays and reduction scratch.
struct Layout {
    int pitch, rows;
    size_t plane, esz;
    size_t off_f[2], off_lo[2], off_T[2], off_mom, off_scr, off_part, off_out, off_stat, total;
};

// Health counters of a channel (unsigned 64-bit, device memory): the two
// the step kernels add to (non-finite readings, psi clamps) and the count
// of non-finite nodes found by the last read-out.
enum { kStatNonfinite = 0, kStatClamps = 1, kStatReadout = 2, kStatWords = 4 };

lbm_status fail(lbm_status st, const char* fmt, ...);
bool make_layout(const lbm_params& p, Layout* L);
lbm_status validate(const lbm_params& p);
// Initial density field (host, Nx*Ny, NULL: uniform rho_v) against the EOS:
// every fluid node needs 0 < b rho below the packing limit and a positive
// Eq. 10 argument 2 (P_EOS - rho/3) / G at its initial temperature.
lbm_status check_initial(const lbm_params& p, const double* rho0);
int default_seg_rows(const lbm_params& p, int rows, int min_rows = 2);
void fill_grid(const lbm_params& p, const Layout& L, int seg_rows, lbmk::Grid& g);
void fill_phys(const lbm_params& p, lbmk::Phys& k);

}  // namespace lbmhost
