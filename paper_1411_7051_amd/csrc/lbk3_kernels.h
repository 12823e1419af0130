// lbk3_kernels.h -- launch interface of the D3Q19 sweep, read-out and
// set-up kernels (lbk3_kernels.hip).  Read-out partials use the MAC_*,
// ST_* and FLD_* slots of the D2Q9 path and its finish kernel.
#pragma once

#include "lbk_kernels.h"

namespace lbk {

constexpr int kBlock3 = 256;

// Lattice extent; rows are (y, z) lines of x, row index z * ny + y; pitch =
// elements per row slot (a multiple of 64).
struct Geom3 {
    int nx, ny, nz, pitch;
};

// The D2Q9 scalars plus the z component of the external acceleration.
struct Physics3 {
    Physics ph;
    float gz;
};

// Blocks of one launch over the lattice (kBlock3 nodes of one row each).
int blocks3_of(const Geom3 &g);

// One step (pull, pressure planes, collide, store) src -> dst.
hipError_t launch_sweep3(int storage, int bcx, int bcy, int bcz, const char *src, char *dst,
                         const Layout &lay, const char *med, const MLayout &mlay,
                         const Geom3 &g, const Physics3 &p3, float s, float inv_s,
                         hipStream_t st);

// Read-out of rho and u ([nz][ny][nx], any may be NULL) and per-block FP64
// partials [MAC_SLOTS][blocks3_of(g)].
hipError_t launch_macro3(int storage, int bcx, int bcy, int bcz, const char *src,
                         const Layout &lay, const char *med, const MLayout &mlay,
                         const Geom3 &g, const Physics3 &p3, float s, float inv_s, float *rho,
                         float *ux, float *uy, float *uz, double *partials, hipStream_t st);

// Mass / max|h| / non-finite partials [ST_SLOTS][blocks].
hipError_t launch_state_sums3(int storage, const char *src, const Layout &lay, const Geom3 &g,
                              float inv_s, double *partials, hipStream_t st);

// Rest state (ramp != 0: linear density ramp rho_in -> rho_out along x).
hipError_t launch_init3(int storage, char *dst, const Layout &lay, const Geom3 &g, int ramp,
                        double rho0, double rho_in, double rho_out, float s, hipStream_t st);

// Post-collision populations in FP64, [19][nz][ny][nx].
hipError_t launch_populations3(int storage, const char *src, const Layout &lay, const Geom3 &g,
                               float inv_s, double *out, hipStream_t st);

// Multiply the stored deviations by 2^k (exact).
hipError_t launch_rescale3(int storage, char *state, const Layout &lay, const Geom3 &g, int k,
                           hipStream_t st);

// Medium validation and k -> drag in place, invalid counts into partials
// [FLD_SLOTS][blocks].
hipError_t launch_fields3(char *med, const MLayout &mlay, const Geom3 &g, double nu,
                          double *partials, hipStream_t st);

} // namespace lbk
