// lbk_adjoint.h -- launch interface of the reverse (adjoint) sweep.
#pragma once

#include "lbk_device.h"
#include "lbk_kernels.h"

namespace lbk {

// One reverse step of the lattice (terminal = 0), or the adjoint of the
// read-out of J = sum_x a1 rho u_x + a2 u_x (terminal = 1; a1 only on column
// nx-1 when outlet = 1).  mu_in / mu_out: adjoint states [y][9][pitch] FP32;
// hist: (rho, jx, jy) [y][pitch][3] of the forward step being reversed;
// grad: FP32 [y][pitch] d J / d ln k, accumulated over a segment; grad2:
// likewise d J / d ln kn0, or NULL to skip that plane.
hipError_t launch_adjoint(int bcx, int bcy, const float *mu_in, float *mu_out, const float *hist,
                          const char *med, const MLayout &mlay, float *grad, float *grad2,
                          const Geom &g, const Physics &ph, int terminal, float a1, float a2,
                          int outlet, hipStream_t st);

// Two reverse steps in one pass, bitwise two launch_adjoint calls (terminal
// = 0) through an intermediate adjoint state that stays in registers:
// mu_in = mu_n -> mu_out = mu_{n-2} (different arrays), hist1 / hist0 the
// histories of steps n and n - 1; rows marched in bands of `band` >= 1.
hipError_t launch_adjoint2(int bcx, int bcy, const float *mu_in, float *mu_out,
                           const float *hist1, const float *hist0, const char *med,
                           const MLayout &mlay, float *grad, float *grad2, const Geom &g,
                           const Physics &ph, int band, hipStream_t st);

// total[y][x] += seg[y][x]; seg[y][x] = 0 ([y][pitch]).
hipError_t launch_grad_fold(float *seg, double *total, const Geom &g, hipStream_t st);

// out[y][x] = (float) grad[y][x] (unpadded [ny][nx]).
hipError_t launch_grad_out(const double *grad, float *out, const Geom &g, hipStream_t st);

// Batched gradients over a batch's tile list (tiles of tile_x by rows, one
// workgroup per tile).  Reverse step: lam_in < 0 is the terminal read-out
// (into lam[0]), else lam[lam_in] -> lam[lam_in ^ 1] with the history in
// hist_slot; kn: also the ln kn0 plane; fc: some sample has the
// Forchheimer term on.
hipError_t launch_batch_adjoint(int bcx, int bcy, const AdjSampleDesc *samples,
                                const int *tile_sample, int ntiles, int tile_x, int rows,
                                int lam_in, int hist_slot, int kn, int fc, hipStream_t st);

// Two reverse steps of every sample of a batched gradient, lam[lam_in] ->
// lam[lam_in ^ 1] (lam_in 0 or 1), histories in slots hist_slot and
// hist_slot - 1 (hist_slot >= 1), over the batch's two-step tiling (tiles of
// four 60-column strips by `band` rows; the descriptors' tile0 / tpr must
// describe it); bitwise two launch_batch_adjoint calls.
hipError_t launch_batch_adjoint2(int bcx, int bcy, const AdjSampleDesc *samples,
                                 const int *tile_sample, int ntiles, int band, int lam_in,
                                 int hist_slot, int kn, int fc, hipStream_t st);

// Gradient planes of every sample: op 0 clears segments and totals, op 1
// folds segments into totals (and clears them), op 2 writes the totals to
// the output planes.
hipError_t launch_batch_grad(const AdjSampleDesc *samples, const int *tile_sample, int ntiles,
                             int tile_x, int rows, int op, int kn, hipStream_t st);

} // namespace lbk
