// lbk_host.h -- host-side internals shared by the C ABI sources (not part of
// the public interface): the lattice handle, its workspace layout, the
// per-thread error message and helpers that sequence launches on the
// handle's stream.
#pragma once

#include "lbk.h"
#include "lbk_kernels.h"

#include <rocprofiler-sdk-roctx/roctx.h>
#include <stddef.h>
#include <stdint.h>

namespace lbk {

// A named roctx range for the lifetime of the object: the phases of a call
// (stepping, checkpointed forward, rebuild, recompute, reverse, graph
// replay) show up as ranges in a rocprofv3 --marker-trace.  Costs a call
// into the roctx library per range, nothing on the device.
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

// Record a formatted message as the calling thread's last error; returns s.
lbk_status fail(lbk_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(LBK_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));             \
    } while (0)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Byte offsets of every region in the workspace, and the strided layouts
// the kernels use.  Each time level of the state is ny row blocks of
// [rho FP32 | h_0 .. h_8 T], each slot `pitch` elements; the medium is ny
// row blocks of [eps | drag | kn0] FP32.
struct WsLayout {
    int pitch;
    Layout lay;           // state row layout
    MLayout mlay;         // medium row layout
    size_t level_bytes;   // bytes of one time level
    size_t level[2];      // two time levels
    size_t med, uxp, uyp; // medium; previous velocity for the residual
    size_t partials, results;
    size_t total;
    int blocks;
};

// Byte offsets of an adjoint workspace for (n, c1, c2): outer checkpoints
// every c1 steps, inner checkpoints every c2 steps (two-level only), two
// recompute levels, c2 + 1 history slots (c1 + 1 for one level), two
// adjoint states, the FP32 per-segment gradient and its FP64 total.
struct AdjPlan {
    bool valid;
    int objective;
    int64_t n, c1, c2, t0;
    bool two_level;
    int64_t k1, k2, hlen;
    int64_t keep; // trailing outer segments whose inner checkpoints the forward keeps
    size_t outer, inner, rec, hist, lam, grad, seg, grad2, seg2, total;
    size_t inner_seg; // bytes of one segment's inner checkpoints (k2 levels)
    size_t level_bytes, hist_bytes, lam_bytes;
    const void *ws;
    double a1, a2;
    int outlet;
};

} // namespace lbk

struct lbk_lattice {
    using WsLayout = lbk::WsLayout;
    using AdjPlan = lbk::AdjPlan;
    using Geom = lbk::Geom;
    using Physics = lbk::Physics;
    lbk_desc d;
    WsLayout L;
    Geom g;
    Physics ph;
    hipStream_t stream;
    int device;    // the HIP device current at create
    char *ws;
    int cur;       // time level holding the current state
    int64_t t;     // steps taken
    uint64_t version; // bumped by every change of the state (steps, loads,
                      // rescaling), so a batch can tell that its cached
                      // tables and read-out sums no longer describe it
    int scale_exp; // FP16: stored = h * 2^scale_exp
    bool have_prev;
    double eps_b;  // mean porosity of the two pressure columns
    double *host;  // pinned scratch for results (8 doubles)
    AdjPlan adj;

    char *state(int l) const { return ws + L.level[l]; }
    char *med() const { return ws + L.med; }
    float s() const { return ldexpf(1.0f, scale_exp); }
    float inv_s() const { return ldexpf(1.0f, -scale_exp); }
    double *partials() const { return reinterpret_cast<double *>(ws + L.partials); }
    double *results() const { return reinterpret_cast<double *>(ws + L.results); }
};

namespace lbk {

// Rows per band of the two-step sweep, by storage.  Short bands keep the
// waves that run at once on nearby rows (a band of 8 recomputes 2 of every
// 10 intermediate rows, yet FP32 measured fastest at 6 to 8 on a 4096 x 4096
// lattice: tall bands spread the concurrent accesses over the whole level
// and ran up to 25% slower); FP16 and BF16, with half the bytes per row,
// measured fastest at 10 to 12.
#ifndef LBK_BAND2
#define LBK_BAND2 8
#endif
#ifndef LBK_BAND2_HALF
#define LBK_BAND2_HALF 10
#endif
inline int band2_of(int storage) { return storage == LBK_F32 ? LBK_BAND2 : LBK_BAND2_HALF; }
// Rows per band of the three-step pass: FP32 ran at 117.7 / 119.6 / 122.5 /
// 121.7 / 117.3 GLUPS with bands of 8 / 10 / 12 / 16 / 24 rows on the
// 4096 x 4096 disc medium; FP16 at 119.5 / 125.1 / 126.9 / 127.4 with 8 /
// 12 / 20 / 24 (BF16 alike).
#ifndef LBK_BAND3
#define LBK_BAND3 12
#endif
#ifndef LBK_BAND3_HALF
#define LBK_BAND3_HALF 24
#endif
inline int band3_of(int storage) { return storage == LBK_F32 ? LBK_BAND3 : LBK_BAND3_HALF; }
// Rows per band of the two-step reverse pass.
#ifndef LBK_BANDA
#define LBK_BANDA 16
#endif
constexpr int kBandA = LBK_BANDA;

// Waves a two-step pass should at least have: two rounds of the 256 compute
// units at three waves per SIMD, with some to spare.
constexpr int64_t kMinWaves2 = 8192;

// The band of a two-step pass over an nx x ny lattice: `band`, halved (down
// to 2) while the pass would have fewer than kMinWaves2 waves.  On a
// 2048 x 1024 lattice bands of 4 or 2 rows ran at 85-86 GLUPS against 78
// with 8 (and 64 with single sweeps).
inline int band_for(int nx, int ny, int band, int strip = kStrip2)
{
    const int64_t strips = (nx + strip - 1) / strip;
    while (band > 2 && strips * ((ny + band - 1) / band) < kMinWaves2)
        band = (band + 1) / 2;
    return band;
}

// Bands of a lattice's forward and reverse two-step passes: the
// descriptor's band, else by size and storage.
inline int fwd_band(const lbk_desc &d)
{
    return d.band > 0 ? d.band : band_for(d.nx, d.ny, band2_of(d.storage));
}
inline int rev_band(const lbk_desc &d) { return d.band > 0 ? d.band : band_for(d.nx, d.ny, kBandA); }
inline int fwd_band3(const lbk_desc &d)
{
    return d.band > 0 ? d.band : band_for(d.nx, d.ny, band3_of(d.storage), kStrip3);
}

// Lattices from this many nodes on take two-step passes under
// LBK_PASS_AUTO.  Below it too few waves run to hide the march's latency,
// and a level fits the 256 MB on-package cache, so single sweeps are not
// bound by HBM: FP32 on 1024 x 512, 52 GLUPS with single sweeps, 48-51 with
// two-step passes; on 1024 x 1024, 61 against 70.  FP16 and BF16, whose
// single sweeps move half the bytes, switch later: 93 against 85 GLUPS on
// 2048 x 1024, 104 against 111 on 2048 x 2048.
inline int64_t two_step_nodes(int storage)
{
    return storage == LBK_F32 ? (int64_t)1 << 20 : (int64_t)1 << 22;
}
// The same for a batch, counting the nodes of all its samples.  Batches keep
// their bands at band2_of and their samples are often small, with more strip
// and band edges per node, so they switch later; lbk_batch_autotune times
// both passes and settles it per batch.
constexpr int64_t kTwoStepBatchNodes = (int64_t)1 << 22;

// Whether steps of this lattice go through the two-step pass (and the
// reverse steps of its gradients through the two-step reverse pass), as
// pass_mode asks.
inline bool two_step_pass(const lbk_lattice *lat)
{
    const lbk_desc &d = lat->d;
    return d.pass_mode == LBK_PASS_TWO_STEP || d.pass_mode == LBK_PASS_THREE_STEP ||
           (d.pass_mode == LBK_PASS_AUTO && (int64_t)d.nx * d.ny >= two_step_nodes(d.storage));
}

// Lattices from this many nodes on take three-step passes under
// LBK_PASS_AUTO.  FP32, against two-step passes: 116.1 against 88.9 GLUPS on
// 4096 x 2048, 95.6 against 82.0 on 2048 x 2048, but 81.3 against 93.6 on
// 2048 x 1024.  FP16: 126.0 against 118.3 on 4096 x 2048, but 104.5 against
// 110.7 on 2048 x 2048 (bands of 24 rows, shortened there to keep the
// device filled).
inline int64_t three_step_nodes(int storage)
{
    return storage == LBK_F32 ? (int64_t)1 << 22 : (int64_t)1 << 23;
}

// Whether lbk_step advances this lattice three steps per launch (so do its
// gradients' rebuilding and recording passes; the reverse passes take two).
inline bool three_step_pass(const lbk_lattice *lat)
{
    const lbk_desc &d = lat->d;
    return d.pass_mode == LBK_PASS_THREE_STEP ||
           (d.pass_mode == LBK_PASS_AUTO && (int64_t)d.nx * d.ny >= three_step_nodes(d.storage));
}

// n >= 0 steps of the lattice on stream st (pairs through the two-step
// sweep); advances time and version.
lbk_status advance(lbk_lattice *lat, int64_t n, hipStream_t st);

// Finish kernel over the handle's partials, `slots` doubles into lat->host
// (synchronizes the stream).
lbk_status fetch(lbk_lattice *lat, int slots, unsigned max_mask);

// NaN/Inf check of the current state; FP16 also re-centres the scale.
lbk_status check_state(lbk_lattice *lat);

// Read-out sums (MAC_* slots) of the current state into lat->host.
lbk_status macro_sums(lbk_lattice *lat, bool residual);

// Whether the run has a drive the global permeability is normalised by: a
// pressure difference (pressure columns) or a body force along x.
bool has_drive(const lbk_desc &d);

// Global permeability (Sec. IV.A, Darcy's law) from read-out sums
// (MAC_* slots over every node); NaN without a drive.
double k_app_of(const lbk_lattice *lat, const double *sums);

// Workspace offsets of a gradient over n steps, checkpoints every c1,
// history c2 at a time (1 <= c2 <= c1).  The inner checkpoints come last:
// the minimum (total) holds those of one segment; with ws_bytes >= total,
// adj_keep sets how many trailing segments' inner checkpoints fit (keep)
// and the bytes they use.
lbk_status adj_plan(const lbk_lattice *lat, int64_t n, int64_t c1, int64_t c2, AdjPlan &P);
void adj_keep(AdjPlan &P, size_t ws_bytes);
// Plain sweeps the backward pass spends rebuilding inner checkpoints.
int64_t adj_rebuild_steps(const AdjPlan &P);

// Gradients need a known objective and, for the global permeability, a drive
// it can be normalised by.
lbk_status check_objective(const lbk_lattice *lat, int objective);

// J from read-out sums, and its per-node weights: J = sum a1 rho u_x +
// a2 u_x (a1 on column nx-1 only when outlet).
double objective_weights(const lbk_lattice *lat, int objective, const double *sums, double &a1,
                         double &a2, int &outlet);

} // namespace lbk
