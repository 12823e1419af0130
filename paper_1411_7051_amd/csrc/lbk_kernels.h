// lbk_kernels.h -- launch interface between the C-ABI host code and the HIP
// kernels of the Klinkenberg lattice Boltzmann sweep.
#pragma once

#include "lbk_device.h"

namespace lbk {

// Threads per block of every lattice kernel: one node per thread, blocks
// cover 256 consecutive x of one row.
constexpr int kBlock = 256;

// Launch geometry of the lattice kernels (1-D grid, XCD-aware remap).
struct Launch {
    int blocks_per_row; // ceil(nx / kBlock)
    int blocks;         // blocks_per_row * ny
};

Launch launch_of(const Geom &g);

// Columns a wave of the two-step pass stores (its strip; the wave's other
// four lanes hold halo columns).
constexpr int kStrip2 = 60;
// Columns a wave of the three-step pass stores (six halo lanes).
constexpr int kStrip3 = 58;

// Largest batch tile width (workgroup size) of the batched sweep.
constexpr int kBatchMaxTile = 256;

// One sample of a batch: its two time levels, medium, layouts, scalars and
// FP16 scale, and where its tiles sit in the batch's tile list (tile0, and
// tiles per tile row across x).
struct SampleDesc {
    char *state[2];
    const char *med;
    Layout lay;
    MLayout mlay;
    Geom g;
    Physics ph;
    float s, inv_s;
    int tile0, tpr;
};

// Slots of the FP64 block partials written by the reduction kernels.
enum {
    MAC_FLUX = 0, // sum rho u_x
    MAC_UX,       // sum u_x
    MAC_DU2,      // sum |u - u_prev|^2
    MAC_U2,       // sum |u|^2
    MAC_RHO,      // sum rho
    MAC_QOUT,     // sum over column nx-1 of rho u_x (outlet mass flux)
    MAC_SLOTS
};
enum {
    ST_MASS = 0,  // sum over nodes of sum_i f*_i
    ST_HMAX,      // max |h_i| (unscaled)
    ST_BAD,       // number of non-finite stored values
    ST_SLOTS
};
enum {
    FLD_BAD = 0,  // number of invalid field values
    FLD_SLOTS
};

// One sweep src -> dst; if hist is non-null also write this step's
// linearisation point (rho, jx, jy) as [y][pitch][3] FP32 for the adjoint.
hipError_t launch_sweep(int storage, int bcx, int bcy, const char *src, char *dst,
                        const Layout &lay, const char *med, const MLayout &mlay, const Geom &g,
                        const Physics &ph, float s, float inv_s, float *hist, hipStream_t st);

// Two steps src -> dst in one pass (bitwise the result of two launch_sweep
// calls through an intermediate level), the old and intermediate levels
// held in registers: waves own strips of 60 columns and march along bands of
// `band` >= 1 rows.  src and dst must be different levels.  With hist1 and
// hist2 (both or neither) the two steps' linearisation points are recorded
// as launch_sweep records one.
hipError_t launch_sweep2(int storage, int bcx, int bcy, const char *src, char *dst,
                         const Layout &lay, const char *med, const MLayout &mlay, const Geom &g,
                         const Physics &ph, float s, float inv_s, int band, float *hist1,
                         float *hist2, hipStream_t st);

// Three steps src -> dst in one pass (bitwise the result of three
// launch_sweep calls), the old level and two intermediate levels held in
// registers: waves own strips of 58 columns and march along bands of
// `band` >= 1 rows.  src and dst must be different levels.  With hist1..3
// (all or none) the three steps' linearisation points are recorded as
// launch_sweep records one.
hipError_t launch_sweep3x(int storage, int bcx, int bcy, const char *src, char *dst,
                          const Layout &lay, const char *med, const MLayout &mlay, const Geom &g,
                          const Physics &ph, float s, float inv_s, int band, float *hist1,
                          float *hist2, float *hist3, hipStream_t st);

// Macroscopic read-out ([ny][nx] outputs, any may be null) and FP64 partials
// [MAC_SLOTS][blocks].  If u_prev ([ny][pitch]) is given it is read for the
// residual and then overwritten with the current velocity.
hipError_t launch_macro(int storage, int bcx, int bcy, const char *src, const Layout &lay,
                        const char *med, const MLayout &mlay, const Geom &g, const Physics &ph,
                        float s, float inv_s, float *rho_out, float *ux_out, float *uy_out,
                        float *ux_prev, float *uy_prev, double *partials, hipStream_t st);

// The read-out sums of launch_macro (no outputs, no residual) over a fixed
// grid of `grid` workgroups that walk the lattice: partials
// [MAC_SLOTS][grid].
hipError_t launch_macro_strided(int storage, int bcx, int bcy, const char *src,
                                const Layout &lay, const char *med, const MLayout &mlay,
                                const Geom &g, const Physics &ph, float s, float inv_s, int grid,
                                double *partials, hipStream_t st);

// Mass / max|h| / non-finite partials [ST_SLOTS][blocks] of a state.
hipError_t launch_state_sums(int storage, const char *src, const Layout &lay, const Geom &g,
                             float inv_s, double *partials, hipStream_t st);

// Reduce partials [slots][blocks] in a fixed order into out[slots]; bit k of
// max_mask selects max instead of sum for slot k.
hipError_t launch_finish(const double *partials, int slots, int blocks, unsigned max_mask,
                         double *out, hipStream_t st);

// Field set-up: in place, turn the raw k slot into drag = eps nu / k
// (0 where k = +inf or eps = 0) and count invalid values into
// partials [FLD_SLOTS][blocks].
hipError_t launch_fields(char *med, const MLayout &mlay, const Geom &g, double nu,
                         double *partials, hipStream_t st);

// Initial state at rest: rho = rho0, or the linear ramp rho_in -> rho_out.
hipError_t launch_init_state(int storage, char *dst, const Layout &lay, const Geom &g, int ramp,
                             double rho0, double rho_in, double rho_out, float s,
                             hipStream_t st);

// FP64 reconstruction f*_i = w_i rho + h_i / s into out[9][ny][nx].
hipError_t launch_populations(int storage, const char *src, const Layout &lay, const Geom &g,
                              float inv_s, double *out, hipStream_t st);

// Multiply every stored deviation by 2^k (FP16 scale re-centring; exact).
hipError_t launch_rescale(int storage, char *state, const Layout &lay, const Geom &g, int k,
                          hipStream_t st);

// One sample of a batched gradient: its levels (the lattice's current level
// and, in its adjoint workspace, the outer / inner checkpoint and recompute
// level arrays, level_bytes apart), history slots, adjoint states, FP32
// segment and FP64 total gradient planes (the second plane is ln kn0), the
// read-out weights of J, the output planes, and its tiles in the batch's
// tile list.
enum { ADJ_CUR = 0, ADJ_OUTER = 1, ADJ_INNER = 2, ADJ_REC = 3 };
struct AdjSampleDesc {
    char *region[4];
    uint64_t level_bytes;
    float *hist;
    uint64_t hist_bytes;
    float *lam[2];
    float *seg, *seg2;
    double *grad, *grad2;
    float *out, *out2;
    const char *med;
    Layout lay;
    MLayout mlay;
    Geom g;
    Physics ph;
    float s, inv_s, a1, a2;
    int outlet, tile0, tpr;
};

// A level of a batched gradient's sample: region ADJ_* and index.
struct LevelSel {
    int region, index;
};

// One recomputing step of every sample of a batched gradient: level src ->
// level dst, recording the history into slot hist_slot (< 0: none).  Tiles
// of tile_x by rows, one workgroup per tile.
hipError_t launch_batch_rec_sweep(int storage, int bcx, int bcy, const AdjSampleDesc *samples,
                                  const int *tile_sample, int ntiles, int tile_x, int rows,
                                  LevelSel src, LevelSel dst, int hist_slot, hipStream_t st);

// Two recomputing steps of every sample of a batched gradient in one pass
// (bitwise two launch_batch_rec_sweep calls): level src -> dst, recording
// into history slots hist_slot and hist_slot + 1 (hist_slot < 0: none),
// over the batch's two-step tiling (see launch_batch_sweep2).
hipError_t launch_batch_rec_sweep2(int storage, int bcx, int bcy, const AdjSampleDesc *samples,
                                   const int *tile_sample, int ntiles, int band, LevelSel src,
                                   LevelSel dst, int hist_slot, hipStream_t st);

// One step of every sample of a batch, parity -> parity ^ 1, over tiles of
// tile_x (a multiple of 64 up to kBatchMaxTile: the workgroup size) by rows
// nodes; the descriptors' tile0/tpr must describe that tiling.  grid > 0:
// persistent launch of grid workgroups each sweeping a contiguous tile
// range; 0: one workgroup per tile.
hipError_t launch_batch_sweep(int storage, int bcx, int bcy, const SampleDesc *samples,
                              const int *tile_sample, int ntiles, int parity, int tile_x,
                              int rows, int grid, hipStream_t st);

// Two-step pass of every sample of a batch, parity -> parity ^ 1: tiles of
// four 60-column strips by `band` rows, one workgroup (kBlock) per tile, in
// the band-major order of the single-lattice pass; the descriptors'
// tile0/tpr must describe that tiling (tpr = groups of four strips per
// band).
hipError_t launch_batch_sweep2(int storage, int bcx, int bcy, const SampleDesc *samples,
                               const int *tile_sample, int ntiles, int parity, int band,
                               hipStream_t st);

// Read-out partials of every sample over tiles of kBlock nodes
// ([MAC_SLOTS][ntiles]) and their per-sample fixed-order sums
// out[nsamples][slots].
hipError_t launch_batch_macro(int storage, int bcx, int bcy, const SampleDesc *samples,
                              const int *tile_sample, int ntiles, int parity, double *partials,
                              hipStream_t st);
hipError_t launch_batch_finish(const SampleDesc *samples, int nsamples, const double *partials,
                               int slots, int ntiles, double *out, hipStream_t st);

} // namespace lbk
