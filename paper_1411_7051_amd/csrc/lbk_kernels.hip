// lbk_kernels.hip -- HIP kernels (gfx950) of the Klinkenberg lattice
// Boltzmann hot path: the fused pull-stream + Klinkenberg + velocity +
// BGK/Guo collide sweep (one launch per time step, Eq. 12), the macroscopic
// read-out (Eqs. 16-17), deterministic FP64 reductions for the global
// permeability and mass, and field / state set-up.
//
// Layout in HBM.  One time level of the state is a stack of row blocks;
// row block y holds, for x = 0 .. pitch-1,
//     rho   FP32      node density
//     h_0 .. h_8  T   deviations f*_i - w_i rho   (T = FP32, FP16 or BF16)
// so one step's reads of rows y-1, y, y+1 and writes of row y stay within a
// few hundred KiB of each other (DRAM page locality), instead of spreading
// over ten planes hundreds of MiB apart.  Two levels ping-pong.  The
// read-only medium (eps, drag = eps nu / k, kn0; FP32) is row-interleaved
// the same way.
//
// Work mapping: one node per thread, 256 threads = 4 wave64s per block, a
// block covers 256 consecutive x of one row, so row pointers are uniform.
// The 1-D grid is remapped so that each of the 8 XCDs (which receive blocks
// round-robin) sweeps one contiguous band of rows: neighbouring rows share
// the density in that XCD's L2.
#include "lbk_kernels.h"

namespace lbk {

Launch launch_of(const Geom &g)
{
    Launch l;
    l.blocks_per_row = (g.nx + kBlock - 1) / kBlock;
    l.blocks = l.blocks_per_row * g.ny;
    return l;
}

// Hardware block b lands on XCD b % 8; give XCD j the j-th contiguous chunk
// of logical blocks.  A bijection on [0, nb) for any nb.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int j = b & 7, idx = b >> 3;
    return j * q + (j < r ? j : r) + idx;
}

// Row and column of this thread's node; y is uniform across the block.
struct Node {
    int y;
    uint32_t x;
    int L; // logical block index
};
__device__ __forceinline__ Node node_of(int bpr)
{
    Node n;
    n.L = xcd_remap(blockIdx.x, gridDim.x);
    n.y = n.L / bpr;
    n.x = (uint32_t)(n.L - n.y * bpr) * kBlock + threadIdx.x;
    return n;
}

// Medium of row y: eps, drag and kn0 at x.
struct Med {
    Rsrc r;
    uint32_t slot, slot2; // byte offsets of the drag and kn0 slots
    __device__ __forceinline__ float eps(uint32_t x) const { return ld_f32(r, x * 4, 0); }
    __device__ __forceinline__ float drag(uint32_t x) const { return ld_f32(r, x * 4, slot); }
    __device__ __forceinline__ float kn0(uint32_t x) const { return ld_f32(r, x * 4, slot2); }
};

// Pressure-column override (non-equilibrium extrapolation from the
// neighbouring column): on entry d, rho, inc, r are the neighbour's pulled
// deviations, density and density residual and en, dragn, kn0n its medium;
// on return d holds the boundary node's deviations relative to the imposed
// density rb (returned), inc = 0 and r its density residual:
//   f_i = f_eq_i(rho_b, u_n; eps_b) + f_i(n) - f_eq_i(rho_n, u_n; eps_n)
template <typename T>
__device__ __forceinline__ float extrapolate(const Physics &ph, float s, float inv_s, bool in,
                                             float eb, float en, float dragn, float kn0n,
                                             float rho, float (&d)[9], float &inc, float &r)
{
    float jx, jy, ux, uy, Fx, Fy;
    momentum(d, jx, jy);
    if (Elem<T>::kScaled) {
        jx *= inv_s;
        jy *= inv_s;
    }
    velocity(ph, rho, jx, jy, en, dragn, kn0n, ux, uy, Fx, Fy);
    const float rb = in ? ph.rin_hi : ph.rout_hi;
    const float rbl = in ? ph.rin_lo : ph.rout_lo;
    // f_eq_i(rho_b, u; eps_b) - f_eq_i(rho_n, u; eps_n) of Eq. 14 as
    // w_i [a e.u + b (4.5 (e.u)^2 - 1.5 u.u)], each equilibrium's
    // deviation from w_i rho vanishing at eps = 0
    const bool sb = !(eb > 0.0f), sn = !(en > 0.0f);
    const float a = 3.0f * ((sb ? 0.0f : rb) - (sn ? 0.0f : rho));
    const float b = (sb ? 0.0f : rb * __builtin_amdgcn_rcpf(eb)) -
                    (sn ? 0.0f : rho * __builtin_amdgcn_rcpf(en));
    const float uu = ux * ux + uy * uy;
    const float c = (rbl - r) - inc; // w_i (rbl - r) - w_i inc, over w_i
    float sum = 0.0f;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        // physical deviation of the boundary node from w_i rb
        const float eu = edot(ex_of(i), ey_of(i), 0, ux, uy, 0.0f);
        const float q = c + b * (4.5f * eu * eu - 1.5f * uu) + a * eu;
        const float v = w_of(i) * q + (Elem<T>::kScaled ? d[i] * inv_s : d[i]);
        sum += v;
        d[i] = Elem<T>::kScaled ? v * s : v;
    }
    inc = 0.0f;
    r = sum;
    return rb;
}

// Post-stream deviations d_i (storage unit) of node (x, y) after the
// boundary override, relative to rho - inc; returns the FP32 density rho
// and sets inc and the density residual r (physical unit).  A pressure-
// column node pulls at its neighbour xn with the same code as every other
// lane, so that only the extrapolation itself diverges (narrow samples of
// a batch have boundary lanes in a large share of their waves).
template <typename T, int BCX>
__device__ __forceinline__ float post_stream(const Rows &R, const Layout &L, const Med &md,
                                             const Geom &g, const Physics &ph, float s,
                                             float inv_s, uint32_t x, float (&d)[9], float &inc,
                                             float &r)
{
    const bool bnode = BCX == BC_PRESSURE && (x == 0 || x == (uint32_t)g.nx - 1);
    const uint32_t xs = !bnode ? x : (x == 0 ? 1u : (uint32_t)g.nx - 2);
    float rc;
    pull<T, BCX>(R, L, g, s, xs, rc, d);
    const float rho = density<T>(rc, d, inv_s, inc, r);
    if (BCX == BC_PRESSURE && bnode) {
        const float en = md.eps(xs), eb = md.eps(x);
        return extrapolate<T>(ph, s, inv_s, x == 0, eb, en, md.drag(xs), md.kn0(xs), rho, d, inc,
                              r);
    }
    return rho;
}

// Linearisation point (rho, jx, jy) of one step at node (x, y) into a
// history slot [y][pitch][3] (FP32, the node's three values together), for
// the adjoint; nt: streaming stores.
__device__ __forceinline__ void record(float *hist, const Geom &g, int y, uint32_t x, float rho,
                                       float jx, float jy, bool nt = true)
{
    const uint32_t hrow = 3u * (uint32_t)g.pitch * 4u;
    const Rsrc hr = make_rsrc(reinterpret_cast<char *>(hist) + (uint64_t)y * hrow, hrow);
    if (nt)
        st_hist<kNT>(hr, x * 12, rho, jx, jy);
    else
        st_hist<0>(hr, x * 12, rho, jx, jy);
}

// Full update of node (x, y): pull, boundary override, moments, velocity,
// collide, store; with HIST also the step's linearisation point.
template <typename T, int BCX, int BCY, bool HIST>
__device__ __forceinline__ void sweep_node(const char *src, char *dst, const Layout &lay,
                                           const char *med, const MLayout &mlay, const Geom &g,
                                           const Physics &ph, float s, float inv_s, float *hist,
                                           int y, uint32_t x)
{
    const Rows R = rows_of<BCY>(src, lay, g, y);
    const Med md{med_row(med, mlay, y), mlay.slot, 2 * mlay.slot};
    float d[9], inc, r;
    const float rho = post_stream<T, BCX>(R, lay, md, g, ph, s, inv_s, x, d, inc, r);
    float jx, jy, ux, uy, Fx, Fy;
    momentum(d, jx, jy);
    if (Elem<T>::kScaled) {
        jx *= inv_s;
        jy *= inv_s;
    }
    if (HIST)
        record(hist, g, y, x, rho, jx, jy);
    const float eps = md.eps(x);
    velocity(ph, rho, jx, jy, eps, md.drag(x), md.kn0(x), ux, uy, Fx, Fy);
    float hs[9];
    collide<T>(ph, rho, inc, r, d, ux, uy, Fx, Fy, eps, s, hs);
    const Rsrc out = make_rsrc(dst + (uint64_t)y * lay.row, (uint32_t)lay.row);
    st_f32(out, x * 4, 0, rho, true);
    constexpr uint32_t es = sizeof(T);
#pragma unroll
    for (int i = 0; i < 9; ++i)
        Elem<T>::st(out, x * es, lay.h_off + i * lay.h_slot, hs[i]);
}

template <typename T, int BCX, int BCY, bool HIST>
__global__ __launch_bounds__(kBlock) void sweep_kernel(const char *src, char *dst, Layout lay,
                                                        const char *med, MLayout mlay, Geom g,
                                                        Physics ph, float s, float inv_s,
                                                        float *hist, int bpr)
{
    const Node nd = node_of(bpr);
    if (nd.x >= (uint32_t)g.nx)
        return;
    sweep_node<T, BCX, BCY, HIST>(src, dst, lay, med, mlay, g, ph, s, inv_s, hist, nd.y, nd.x);
}

// ------------------------------------------------------ two steps a pass
//
// sweep2_kernel advances the lattice by two time steps in one pass, with the
// old level and the intermediate level both held in registers: per node and
// two steps the state is read once and written once.  Each wave owns a strip
// of kStrip2 consecutive columns and a band of rows and marches along y; its
// 64 lanes hold the strip's columns and two more on either side.  Three rows
// of the old level (each loaded once) feed the first step of one
// intermediate row; three intermediate rows feed the second step of one row,
// which is stored.  The x-neighbours of a pull come from the adjacent lanes
// through whole-wave DPP shifts, so each step loses one column on either
// side: the old level is complete on lanes 0..63, the intermediate level on
// lanes 1..62 and the result on lanes 2..61.  Both steps are the single-step
// node update with the neighbour values taken from registers instead of
// HBM, and the intermediate values are rounded to the storage type exactly as
// a store and a reload would round them, so the result is bitwise that of two
// single sweeps.  The four halo columns of each strip and the halo rows at
// each band's ends are computed by the neighbouring strips and bands too.

// One node of a level as a pull reads it: density and deviations (storage
// unit, as stored), with the node's medium.
struct Mid {
    float rho, h[9];
    float eps, drag, kn0;
};

// Node (x, y) of a stored level and its medium.  A row the march loads
// ahead but will not use (live = false, uniform) gets empty buffer
// resources: its loads return 0 without touching memory.
template <typename T>
__device__ __forceinline__ void load_node(const char *src, const Layout &lay, const char *med,
                                          const MLayout &mlay, int y, uint32_t x, Mid &m,
                                          bool live = true)
{
    const Rsrc row = make_rsrc(src + (uint64_t)y * lay.row, live ? (uint32_t)lay.row : 0u);
    // default cache policy: a strip's 64-column loads share their first and
    // last cache lines with the neighbouring strips, which read them about
    // the same time (nontemporal loads fetched those lines twice)
    m.rho = ld_f32(row, x * 4, 0);
    constexpr uint32_t es = sizeof(T);
#pragma unroll
    for (int i = 0; i < 9; ++i)
        m.h[i] = Elem<T>::template ld<0>(row, x * es, lay.h_off + i * lay.h_slot);
    const Rsrc mr = make_rsrc(med + (uint64_t)y * mlay.row, live ? (uint32_t)mlay.row : 0u);
    m.eps = ld_f32(mr, x * 4, 0);
    m.drag = ld_f32(mr, x * 4, mlay.slot);
    m.kn0 = ld_f32(mr, x * 4, 2 * mlay.slot);
}

// The pull of this lane's node from the rows y - 1 (dn), y (c) and y + 1 (up)
// of the previous level: the arithmetic of pull() with the neighbour values
// taken from registers and adjacent lanes.
template <typename T, int BCX>
__device__ __forceinline__ void pull_mid(const Mid &dn, const Mid &c, const Mid &up, bool wym,
                                         bool wyp, bool wxm, bool wxp, float s, float &rc,
                                         float (&d)[9])
{
    rc = c.rho;
    d[0] = c.h[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const int ex = ex_of(i), ey = ey_of(i);
        const bool wall_y = (ey == 1 && wym) || (ey == -1 && wyp); // uniform
        const Mid &m = ey == 1 ? dn : (ey == -1 ? up : c);
        const float ws = Elem<T>::kScaled ? w_of(i) * s : w_of(i);
        float rn, h;
        if (ex == 1) {
            rn = lane_from<1>(m.rho);
            h = lane_from<1>(m.h[i]);
        } else if (ex == -1) {
            rn = lane_from<-1>(m.rho);
            h = lane_from<-1>(m.h[i]);
        } else {
            rn = m.rho;
            h = m.h[i];
        }
        // a wall bounces the pull back: a select, not a branch, so that no
        // control flow splits the row's loads from their uses
        if (ey != 0) {
            rn = wall_y ? c.rho : rn;
            h = wall_y ? c.h[opp_of(i)] : h;
        }
        d[i] = ws * (rn - rc) + h;
        if (BCX == BC_WALL) {
            const bool wall_x = (ex == 1 && wxm) || (ex == -1 && wxp); // per lane, edges only
            if (wall_x)
                d[i] = c.h[opp_of(i)];
        }
    }
}

// Lane-dependent facts of a strip: which column a lane holds and what kind.
struct Lanes {
    uint32_t x;     // the lane's column, wrapped (periodic) or clamped
    bool wxm, wxp;  // x walls on either side of the column
    bool bin, bout; // the inlet / outlet pressure column
    bool has_b;     // uniform: the wave may hold a pressure column
};

// One step of this lane's node at row y from three rows of the previous
// level in registers: pull, pressure-column override from the neighbouring
// lane's pull, moments, velocity and collide -- sweep_node's update.
// Returns the new density, the unrounded deviations hs and, for the
// history, (jx, jy).
template <typename T, int BCX>
__device__ __forceinline__ float step_from(const Physics &ph, float s, float inv_s, const Mid &dn,
                                           const Mid &c, const Mid &up, bool wym, bool wyp,
                                           const Lanes &ln, float (&hs)[9], float &jx, float &jy)
{
    float d[9], rc, inc, r;
    pull_mid<T, BCX>(dn, c, up, wym, wyp, ln.wxm, ln.wxp, s, rc, d);
    float en = 0.0f, dragn = 0.0f, kn0n = 0.0f;
    if (BCX == BC_PRESSURE && ln.has_b) {
        // a pressure column pulls at its neighbour: take that lane's pull
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const float lf = lane_from<-1>(d[i]), rf = lane_from<1>(d[i]);
            d[i] = ln.bin ? lf : (ln.bout ? rf : d[i]);
        }
        const float rl = lane_from<-1>(rc), rr = lane_from<1>(rc);
        rc = ln.bin ? rl : (ln.bout ? rr : rc);
        const float el = lane_from<-1>(c.eps), er = lane_from<1>(c.eps);
        const float dl = lane_from<-1>(c.drag), dr = lane_from<1>(c.drag);
        const float kl = lane_from<-1>(c.kn0), kr = lane_from<1>(c.kn0);
        en = ln.bin ? el : er;
        dragn = ln.bin ? dl : dr;
        kn0n = ln.bin ? kl : kr;
    }
    float rho = density<T>(rc, d, inv_s, inc, r);
    if (BCX == BC_PRESSURE && (ln.bin || ln.bout))
        rho = extrapolate<T>(ph, s, inv_s, ln.bin, c.eps, en, dragn, kn0n, rho, d, inc, r);
    momentum(d, jx, jy);
    if (Elem<T>::kScaled) {
        jx *= inv_s;
        jy *= inv_s;
    }
    float ux, uy, Fx, Fy;
    velocity(ph, rho, jx, jy, c.eps, c.drag, c.kn0, ux, uy, Fx, Fy);
    collide<T>(ph, rho, inc, r, d, ux, uy, Fx, Fy, c.eps, s, hs);
    return rho;
}

// First step of row y: the intermediate node as the second step reads it.
template <typename T, int BCX, bool HIST>
__device__ __forceinline__ void first_step(const Physics &ph, float s, float inv_s, const Geom &g,
                                           const Mid &dn, const Mid &c, const Mid &up, bool wym,
                                           bool wyp, const Lanes &ln, int y, float *hist,
                                           bool rec, Mid &m)
{
    float hs[9], jx, jy;
    m.rho = step_from<T, BCX>(ph, s, inv_s, dn, c, up, wym, wyp, ln, hs, jx, jy);
    if (HIST && rec)
        record(hist, g, y, ln.x, m.rho, jx, jy, false);
#pragma unroll
    for (int i = 0; i < 9; ++i)
        m.h[i] = Elem<T>::round(hs[i]);
    m.eps = c.eps;
    m.drag = c.drag;
    m.kn0 = c.kn0;
}

// The two-step pass of one wave: strip `strip` (60 columns) of band `bnd`
// (rows bnd * band ..) of one lattice, marched downwards (DIR = 1: from the
// band's first row) or upwards (DIR = -1: from its last).  Neighbouring
// bands march in opposite directions, so two bands read the rows they share
// (each band's two halo rows on either side) at the same time -- both at
// their start or both at their end -- while the L2 still holds them.
template <typename T, int BCX, int BCY, bool HIST, int DIR>
__device__ __forceinline__ void sweep2_strip_dir(const char *__restrict__ src,
                                                 char *__restrict__ dst, const Layout &lay,
                                                 const char *__restrict__ med,
                                                 const MLayout &mlay, const Geom &g,
                                                 const Physics &ph, float s, float inv_s,
                                                 int band, int bnd, int strip,
                                                 float *__restrict__ hist1,
                                                 float *__restrict__ hist2)
{
    const int lane = (int)(threadIdx.x & 63);
    const int nstrips = (g.nx + kStrip2 - 1) / kStrip2;
    if (strip >= nstrips)
        return; // the whole wave
    // lane l holds column strip * kStrip2 - 2 + l: lanes 2..kStrip2+1 the
    // strip's own columns, two halo columns on either side
    const int xr = strip * kStrip2 - 2 + lane;
    Lanes ln;
    if (BCX == BC_PERIODIC)
        ln.x = (uint32_t)(((xr % g.nx) + g.nx) % g.nx);
    else
        ln.x = (uint32_t)(xr < 0 ? 0 : (xr >= g.nx ? g.nx - 1 : xr)); // beyond: unused copies
    // A pressure column takes its neighbour's pull, which the second step
    // completes on lanes 2..kStrip2+1 only: an outlet column at lane 2 is
    // left to the previous strip, where it sits at lane kStrip2 + 2.
    bool owned = lane >= 2 && lane <= kStrip2 + 1 && xr < g.nx;
    if (BCX == BC_PRESSURE && xr == g.nx - 1)
        owned = lane >= 3 && lane <= kStrip2 + 2;
    ln.wxm = BCX == BC_WALL && ln.x == 0;
    ln.wxp = BCX == BC_WALL && ln.x == (uint32_t)g.nx - 1;
    ln.bin = BCX == BC_PRESSURE && xr == 0;
    ln.bout = BCX == BC_PRESSURE && xr == g.nx - 1;
    ln.has_b = BCX == BC_PRESSURE && (strip == 0 || strip >= nstrips - 2);
    const int y0 = bnd * band, y1 = min(y0 + band, g.ny), nb = y1 - y0;
    // physical row of march position m (positions 0 .. nb - 1 are the band)
    auto Y = [&](int m) { return DIR > 0 ? y0 + m : y1 - 1 - m; };
    auto wrap = [&](int y) { return BCY == BC_PERIODIC ? ((y % g.ny) + g.ny) % g.ny : y; };
    // A row index that always exists.  A row beyond a wall reads the
    // nearest row and its first step is computed from those values all the
    // same (never recorded, and discarded where the pull bounces back), so
    // that no branch splits the march.
    auto held = [&](int y) {
        return BCY == BC_PERIODIC ? wrap(y) : (y < 0 ? 0 : (y >= g.ny ? g.ny - 1 : y));
    };
    auto wall_lo = [&](int y) { return BCY == BC_WALL && y == 0; };
    auto wall_hi = [&](int y) { return BCY == BC_WALL && y == g.ny - 1; };
    // Every lane stores, so that the stores are not inside a branch: a lane
    // that does not own its column repeats the store of the wave's first
    // owning lane (same address, same value).  With no branch around them
    // the compiler counts exactly how many stores follow a prefetched row's
    // loads and waits for those loads alone, not for the stores too.
    const uint64_t om = __builtin_amdgcn_ballot_w64(owned);
    if (om == 0)
        return; // an outlet strip whose only column the previous strip stores
    const int q = (int)__builtin_ctzll(om);
    const uint32_t xq = (uint32_t)__builtin_amdgcn_readlane((int)ln.x, q);
    const uint32_t xst = owned ? ln.x : xq;
    auto same = [&](float v) {
        const float vq = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), q));
        return owned ? v : vq;
    };
    // The steps in march order: p, c, n are the rows at positions m - 1, m,
    // m + 1, which are the physical rows below, at and above (DIR = 1) or
    // above, at and below (DIR = -1).
    auto first = [&](const Mid &p, const Mid &c, const Mid &n, int m, bool rec, Mid &out) {
        const int y = Y(m);
        first_step<T, BCX, HIST>(ph, s, inv_s, g, DIR > 0 ? p : n, c, DIR > 0 ? n : p,
                                 wall_lo(y), wall_hi(y), ln, wrap(y), hist1, rec, out);
    };

    // For the current output position m: old rows at positions m .. m + 2
    // in use, m + 3 and m + 4 in flight (loads are issued two rows ahead of
    // their use, which keeps enough of them outstanding per wave to cover
    // HBM latency), intermediate rows m - 1 .. m + 1 (m0..m2).
    Mid a1, a2, a3, a4, a5, m0, m1, m2;
    load_node<T>(src, lay, med, mlay, held(Y(-2)), ln.x, a4);
    load_node<T>(src, lay, med, mlay, held(Y(-1)), ln.x, a5);
    load_node<T>(src, lay, med, mlay, Y(0), ln.x, a1);
    load_node<T>(src, lay, med, mlay, held(Y(1)), ln.x, a2);
    first(a4, a5, a1, -1, false, m0);
    first(a5, a1, a2, 0, owned, m1);
    load_node<T>(src, lay, med, mlay, held(Y(2)), ln.x, a3);
    load_node<T>(src, lay, med, mlay, held(Y(3)), ln.x, a4, nb >= 2);
    // One output row: u0..u2 are the old rows at positions m .. m + 2, nx
    // receives position m + 4.  The loop below calls it with the five
    // old-row registers in rotated roles, so no loaded value is ever copied
    // (a copy would make the wave wait for its load -- and for the stores
    // issued after it -- at that point rather than at the value's first use).
    auto row = [&](int m, const Mid &u0, const Mid &u1, const Mid &u2, Mid &nx) {
        // the last output row needs old rows up to position nb + 1
        load_node<T>(src, lay, med, mlay, held(Y(m + 4)), ln.x, nx, m + 4 <= nb + 1);
        first(u0, u1, u2, m + 1, owned && m + 1 < nb, m2);
        const int y = Y(m);
        float hs[9], jx, jy;
        const float rho = step_from<T, BCX>(ph, s, inv_s, DIR > 0 ? m0 : m2, m1,
                                            DIR > 0 ? m2 : m0, wall_lo(y), wall_hi(y), ln, hs,
                                            jx, jy);
        if (HIST && owned)
            record(hist2, g, y, ln.x, rho, jx, jy, false);
        const Rsrc out = make_rsrc(dst + (uint64_t)y * lay.row, (uint32_t)lay.row);
        // default cache policy: a strip's 60 columns cover parts of cache
        // lines whose other parts the neighbouring strips write, which L2
        // merges (streaming stores measured 8% slower per pass)
        st_f32(out, xst * 4, 0, same(rho), false);
        constexpr uint32_t es = sizeof(T);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            Elem<T>::template st<0>(out, xst * es, lay.h_off + i * lay.h_slot, same(hs[i]));
        m0 = m1;
        m1 = m2;
    };
    for (int m = 0; m < nb; m += 5) {
        row(m, a1, a2, a3, a5);
        if (m + 1 >= nb)
            break;
        row(m + 1, a2, a3, a4, a1);
        if (m + 2 >= nb)
            break;
        row(m + 2, a3, a4, a5, a2);
        if (m + 3 >= nb)
            break;
        row(m + 3, a4, a5, a1, a3);
        if (m + 4 >= nb)
            break;
        row(m + 4, a5, a1, a2, a4);
    }
}

// The two-step pass of one wave: even bands march downwards, odd upwards.
template <typename T, int BCX, int BCY, bool HIST>
__device__ __forceinline__ void sweep2_strip(const char *__restrict__ src,
                                             char *__restrict__ dst, const Layout &lay,
                                             const char *__restrict__ med, const MLayout &mlay,
                                             const Geom &g, const Physics &ph, float s,
                                             float inv_s, int band, int bnd, int strip,
                                             float *__restrict__ hist1, float *__restrict__ hist2)
{
    if (bnd & 1)
        sweep2_strip_dir<T, BCX, BCY, HIST, -1>(src, dst, lay, med, mlay, g, ph, s, inv_s, band,
                                                bnd, strip, hist1, hist2);
    else
        sweep2_strip_dir<T, BCX, BCY, HIST, 1>(src, dst, lay, med, mlay, g, ph, s, inv_s, band,
                                               bnd, strip, hist1, hist2);
}

template <typename T, int BCX, int BCY, bool HIST>
__global__ __launch_bounds__(kBlock) void sweep2_kernel(const char *__restrict__ src,
                                                         char *__restrict__ dst, Layout lay,
                                                         const char *__restrict__ med,
                                                         MLayout mlay, Geom g, Physics ph,
                                                         float s, float inv_s, int band,
                                                         int groups, float *__restrict__ hist1,
                                                         float *__restrict__ hist2)
{
    // logical block: band-major, four strips (one per wave) per block
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int bnd = L / groups;
    const int strip = (L - bnd * groups) * (kBlock / 64) + (int)(threadIdx.x >> 6);
    sweep2_strip<T, BCX, BCY, HIST>(src, dst, lay, med, mlay, g, ph, s, inv_s, band, bnd, strip,
                                    hist1, hist2);
}

// sweep3x_kernel advances the lattice by three time steps in one pass: the
// two-step pass with a second intermediate level.  A wave's 64 lanes hold a
// strip of kStrip3 columns and three halo columns on either side; the first
// intermediate level is complete on lanes 1..62, the second on 2..61 and
// the result on 3..60, which the strip owns.  Per output row y the wave
// keeps the old rows y + 1 .. y + 3 (y + 4 and y + 5 in flight), the first
// intermediate rows y .. y + 2 and the second y - 1 .. y + 1.  Every
// intermediate level is rounded as a store would round it, so the pass is
// bitwise three single sweeps.  With HIST it records the three steps'
// linearisation points for the adjoint, each row by the band that owns it.
template <typename T, int BCX, int BCY, bool HIST, int DIR>
__device__ __forceinline__ void sweep3x_strip_dir(const char *__restrict__ src,
                                                  char *__restrict__ dst, const Layout &lay,
                                                  const char *__restrict__ med,
                                                  const MLayout &mlay, const Geom &g,
                                                  const Physics &ph, float s, float inv_s,
                                                  int band, int bnd, int strip,
                                                  float *__restrict__ hist1,
                                                  float *__restrict__ hist2,
                                                  float *__restrict__ hist3)
{
    const int lane = (int)(threadIdx.x & 63);
    const int nstrips = (g.nx + kStrip3 - 1) / kStrip3;
    if (strip >= nstrips)
        return; // the whole wave
    // lane l holds column strip * kStrip3 - 3 + l: lanes 3..kStrip3+2 the
    // strip's own columns, three halo columns on either side
    const int xr = strip * kStrip3 - 3 + lane;
    Lanes ln;
    if (BCX == BC_PERIODIC)
        ln.x = (uint32_t)(((xr % g.nx) + g.nx) % g.nx);
    else
        ln.x = (uint32_t)(xr < 0 ? 0 : (xr >= g.nx ? g.nx - 1 : xr)); // beyond: unused copies
    // A pressure column takes its neighbour's pull, which the third step
    // completes on lanes 3..kStrip3+2 only: an outlet column at lane 3 is
    // left to the previous strip, where it sits at lane kStrip3 + 3.
    bool owned = lane >= 3 && lane <= kStrip3 + 2 && xr < g.nx;
    if (BCX == BC_PRESSURE && xr == g.nx - 1)
        owned = lane >= 4 && lane <= kStrip3 + 3;
    ln.wxm = BCX == BC_WALL && ln.x == 0;
    ln.wxp = BCX == BC_WALL && ln.x == (uint32_t)g.nx - 1;
    ln.bin = BCX == BC_PRESSURE && xr == 0;
    ln.bout = BCX == BC_PRESSURE && xr == g.nx - 1;
    ln.has_b = BCX == BC_PRESSURE && (strip == 0 || strip >= nstrips - 2);
    const int y0 = bnd * band, y1 = min(y0 + band, g.ny), nb = y1 - y0;
    auto Y = [&](int m) { return DIR > 0 ? y0 + m : y1 - 1 - m; };
    auto wrap = [&](int y) { return BCY == BC_PERIODIC ? ((y % g.ny) + g.ny) % g.ny : y; };
    // rows beyond a wall: as in the two-step pass, computed from the
    // nearest row and discarded by the bounce-back selects
    auto held = [&](int y) {
        return BCY == BC_PERIODIC ? wrap(y) : (y < 0 ? 0 : (y >= g.ny ? g.ny - 1 : y));
    };
    auto wall_lo = [&](int y) { return BCY == BC_WALL && y == 0; };
    auto wall_hi = [&](int y) { return BCY == BC_WALL && y == g.ny - 1; };
    const uint64_t om = __builtin_amdgcn_ballot_w64(owned);
    if (om == 0)
        return; // an outlet strip whose only column the previous strip stores
    const int q = (int)__builtin_ctzll(om);
    const uint32_t xq = (uint32_t)__builtin_amdgcn_readlane((int)ln.x, q);
    const uint32_t xst = owned ? ln.x : xq;
    auto same = [&](float v) {
        const float vq = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), q));
        return owned ? v : vq;
    };
    // One step of the row at march position m from the rows at m - 1, m,
    // m + 1 of the level below (old or intermediate), rounded as stored;
    // recorded into hist where rec (a row of this band, an owned lane).
    auto step = [&](const Mid &p, const Mid &c, const Mid &n, int m, float *hist, bool rec,
                    Mid &out) {
        const int y = Y(m);
        first_step<T, BCX, HIST>(ph, s, inv_s, g, DIR > 0 ? p : n, c, DIR > 0 ? n : p,
                                 wall_lo(y), wall_hi(y), ln, wrap(y), hist, rec, out);
    };
    auto load = [&](int m, Mid &out) {
        // the last output row needs old rows up to position nb + 2
        load_node<T>(src, lay, med, mlay, held(Y(m)), ln.x, out, m <= nb + 2);
    };

    // old rows a1..a5, first intermediate level p0..p2, second q0..q2
    Mid a1, a2, a3, a4, a5, p0, p1, p2, q0, q1, q2;
    load(-3, a1);
    load(-2, a2);
    load(-1, a3);
    load(0, a4);
    load(1, a5);
    step(a1, a2, a3, -2, hist1, false, p0);
    load(2, a1);
    step(a2, a3, a4, -1, hist1, false, p1);
    load(3, a2);
    step(a3, a4, a5, 0, hist1, owned, p2);
    step(p0, p1, p2, -1, hist2, false, q0);
    load(4, a3);
    p0 = p1;
    p1 = p2;
    step(a4, a5, a1, 1, hist1, owned && 1 < nb, p2);
    step(p0, p1, p2, 0, hist2, owned, q1);
    p0 = p1;
    p1 = p2;
    // One output row m: u1..u3 are the old rows at positions m + 1 .. m + 3,
    // nx receives position m + 5; p0, p1 hold the first level's rows m,
    // m + 1 and q0, q1 the second level's rows m - 1, m.
    auto row = [&](int m, const Mid &u1, const Mid &u2, const Mid &u3, Mid &nx) {
        load(m + 5, nx);
        step(u1, u2, u3, m + 2, hist1, owned && m + 2 < nb, p2);
        step(p0, p1, p2, m + 1, hist2, owned && m + 1 < nb, q2);
        const int y = Y(m);
        float hs[9], jx, jy;
        const float rho = step_from<T, BCX>(ph, s, inv_s, DIR > 0 ? q0 : q2, q1,
                                            DIR > 0 ? q2 : q0, wall_lo(y), wall_hi(y), ln, hs,
                                            jx, jy);
        if (HIST && owned)
            record(hist3, g, y, ln.x, rho, jx, jy, false);
        const Rsrc out = make_rsrc(dst + (uint64_t)y * lay.row, (uint32_t)lay.row);
        st_f32(out, xst * 4, 0, same(rho), false);
        constexpr uint32_t es = sizeof(T);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            Elem<T>::template st<0>(out, xst * es, lay.h_off + i * lay.h_slot, same(hs[i]));
        p0 = p1;
        p1 = p2;
        q0 = q1;
        q1 = q2;
    };
    for (int m = 0; m < nb; m += 5) {
        row(m, a5, a1, a2, a4);
        if (m + 1 >= nb)
            break;
        row(m + 1, a1, a2, a3, a5);
        if (m + 2 >= nb)
            break;
        row(m + 2, a2, a3, a4, a1);
        if (m + 3 >= nb)
            break;
        row(m + 3, a3, a4, a5, a2);
        if (m + 4 >= nb)
            break;
        row(m + 4, a4, a5, a1, a3);
    }
}

template <typename T, int BCX, int BCY, bool HIST>
__global__ __launch_bounds__(kBlock) void sweep3x_kernel(const char *__restrict__ src,
                                                          char *__restrict__ dst, Layout lay,
                                                          const char *__restrict__ med,
                                                          MLayout mlay, Geom g, Physics ph,
                                                          float s, float inv_s, int band,
                                                          int groups, float *__restrict__ hist1,
                                                          float *__restrict__ hist2,
                                                          float *__restrict__ hist3)
{
    // logical block: band-major, four strips (one per wave) per block.  At
    // FP32 neighbouring bands march in opposite directions (122.5 against
    // 117.0 GLUPS marching all one way, 4096 x 4096 discs, bands of 12); the
    // 16-bit passes, bound by instruction issue, march all one way (133.7
    // against 127.4 GLUPS, bands of 24), which halves their code.
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int bnd = L / groups;
    const int strip = (L - bnd * groups) * (kBlock / 64) + (int)(threadIdx.x >> 6);
    if (sizeof(T) == 4 && (bnd & 1))
        sweep3x_strip_dir<T, BCX, BCY, HIST, -1>(src, dst, lay, med, mlay, g, ph, s, inv_s, band,
                                                 bnd, strip, hist1, hist2, hist3);
    else
        sweep3x_strip_dir<T, BCX, BCY, HIST, 1>(src, dst, lay, med, mlay, g, ph, s, inv_s, band,
                                                bnd, strip, hist1, hist2, hist3);
}

// -------------------------------------------------------------- batches
//
// A batch steps many independent lattices (samples of uneven size, each
// with its own layout, medium and scalars) in one launch per step.  The
// work list is the concatenation of every sample's tiles -- blockDim.x
// consecutive x by `rows` consecutive y of one sample -- in sample order,
// tile rows in order; tile_sample maps a tile to its sample.  A workgroup
// reads its tile's descriptor once and sweeps the tile row by row, so the
// dependent descriptor loads are paid once per `rows` rows.
// PERSIST = false: one workgroup per tile, in the XCD-band order of the
// single-lattice kernels.  PERSIST = true: a fixed grid whose workgroup b
// sweeps the contiguous tile range [b T / G, (b + 1) T / G).

template <typename T, int BCX, int BCY>
__device__ __forceinline__ void batch_tile(const SampleDesc *__restrict__ samples,
                                           const int *__restrict__ tile_sample, int rows,
                                           int parity, int t)
{
    // the descriptor is copied before the tile's first store, so its fields
    // stay in scalar registers for every row
    const SampleDesc sd = samples[tile_sample[t]];
    const int rel = t - sd.tile0;
    const int ty = rel / sd.tpr;
    const uint32_t x = (uint32_t)(rel - ty * sd.tpr) * blockDim.x + threadIdx.x;
    if (x >= (uint32_t)sd.g.nx)
        return;
    const char *src = parity ? sd.state[1] : sd.state[0];
    char *dst = parity ? sd.state[0] : sd.state[1];
    const int y0 = ty * rows, y1 = min(y0 + rows, sd.g.ny);
    for (int y = y0; y < y1; ++y)
        sweep_node<T, BCX, BCY, false>(src, dst, sd.lay, sd.med, sd.mlay, sd.g, sd.ph, sd.s,
                                       sd.inv_s, nullptr, y, x);
}

template <typename T, int BCX, int BCY, bool PERSIST>
__global__ __launch_bounds__(kBatchMaxTile) void batch_sweep_kernel(
    const SampleDesc *__restrict__ samples, const int *__restrict__ tile_sample, int ntiles,
    int rows, int parity)
{
    if (PERSIST) {
        const int G = gridDim.x, b = blockIdx.x;
        const int t0 = (int)((int64_t)b * ntiles / G), t1 = (int)((int64_t)(b + 1) * ntiles / G);
        for (int t = t0; t < t1; ++t)
            batch_tile<T, BCX, BCY>(samples, tile_sample, rows, parity, t);
    } else {
        batch_tile<T, BCX, BCY>(samples, tile_sample, rows, parity,
                                xcd_remap(blockIdx.x, gridDim.x));
    }
}

// Two-step pass of every sample of a batch, parity -> parity ^ 1 (two time
// steps): the tile list holds one entry per (sample, band, group of four
// strips); a sample's descriptor gives its first tile and its groups per
// band (tpr).  Each sample's result is bitwise its own two-step pass.
template <typename T, int BCX, int BCY>
__global__ __launch_bounds__(kBlock) void batch_sweep2_kernel(
    const SampleDesc *__restrict__ samples, const int *__restrict__ tile_sample, int band,
    int parity)
{
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const SampleDesc sd = samples[tile_sample[t]];
    const int rel = t - sd.tile0;
    const int bnd = rel / sd.tpr;
    const int strip = (rel - bnd * sd.tpr) * (kBlock / 64) + (int)(threadIdx.x >> 6);
    const char *src = parity ? sd.state[1] : sd.state[0];
    char *dst = parity ? sd.state[0] : sd.state[1];
    sweep2_strip<T, BCX, BCY, false>(src, dst, sd.lay, sd.med, sd.mlay, sd.g, sd.ph, sd.s,
                                     sd.inv_s, band, bnd, strip, nullptr, nullptr);
}

// Recomputing sweep of a batched gradient: the same node update between two
// levels chosen per launch, optionally recording the history.
template <typename T, int BCX, int BCY, bool HIST>
__global__ __launch_bounds__(kBatchMaxTile) void batch_rec_sweep_kernel(
    const AdjSampleDesc *__restrict__ samples, const int *__restrict__ tile_sample, int ntiles,
    int rows, LevelSel src_sel, LevelSel dst_sel, int hist_slot)
{
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const AdjSampleDesc sd = samples[tile_sample[t]];
    const int rel = t - sd.tile0;
    const int ty = rel / sd.tpr;
    const uint32_t x = (uint32_t)(rel - ty * sd.tpr) * blockDim.x + threadIdx.x;
    if (x >= (uint32_t)sd.g.nx)
        return;
    // selects, not an indexed read: the descriptor stays in registers
    auto region = [&](int r) {
        return r == ADJ_CUR ? sd.region[0]
                            : (r == ADJ_OUTER ? sd.region[1]
                                              : (r == ADJ_INNER ? sd.region[2] : sd.region[3]));
    };
    const char *src = region(src_sel.region) + (uint64_t)src_sel.index * sd.level_bytes;
    char *dst = region(dst_sel.region) + (uint64_t)dst_sel.index * sd.level_bytes;
    float *hist = HIST ? reinterpret_cast<float *>(reinterpret_cast<char *>(sd.hist) +
                                                   (uint64_t)hist_slot * sd.hist_bytes)
                       : nullptr;
    const int y0 = ty * rows, y1 = min(y0 + rows, sd.g.ny);
    for (int y = y0; y < y1; ++y)
        sweep_node<T, BCX, BCY, HIST>(src, dst, sd.lay, sd.med, sd.mlay, sd.g, sd.ph, sd.s,
                                      sd.inv_s, hist, y, x);
}

// Two recomputing steps of every sample of a batched gradient in one pass:
// level src -> level dst, recording the two steps' histories into slots
// hist_slot and hist_slot + 1 (hist_slot < 0: none); the batch's two-step
// tiling.
template <typename T, int BCX, int BCY, bool HIST>
__global__ __launch_bounds__(kBlock) void batch_rec_sweep2_kernel(
    const AdjSampleDesc *__restrict__ samples, const int *__restrict__ tile_sample, int band,
    LevelSel src_sel, LevelSel dst_sel, int hist_slot)
{
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const AdjSampleDesc sd = samples[tile_sample[t]];
    const int rel = t - sd.tile0;
    const int bnd = rel / sd.tpr;
    const int strip = (rel - bnd * sd.tpr) * (kBlock / 64) + (int)(threadIdx.x >> 6);
    auto region = [&](int r) {
        return r == ADJ_CUR ? sd.region[0]
                            : (r == ADJ_OUTER ? sd.region[1]
                                              : (r == ADJ_INNER ? sd.region[2] : sd.region[3]));
    };
    const char *src = region(src_sel.region) + (uint64_t)src_sel.index * sd.level_bytes;
    char *dst = region(dst_sel.region) + (uint64_t)dst_sel.index * sd.level_bytes;
    char *h = reinterpret_cast<char *>(sd.hist);
    float *hist1 = HIST ? reinterpret_cast<float *>(h + (uint64_t)hist_slot * sd.hist_bytes)
                        : nullptr;
    float *hist2 = HIST ? reinterpret_cast<float *>(h + (uint64_t)(hist_slot + 1) * sd.hist_bytes)
                        : nullptr;
    sweep2_strip<T, BCX, BCY, HIST>(src, dst, sd.lay, sd.med, sd.mlay, sd.g, sd.ph, sd.s,
                                    sd.inv_s, band, bnd, strip, hist1, hist2);
}

// ----------------------------------------------------------- reductions

struct SumOp {
    static __device__ __forceinline__ double f(double a, double b) { return a + b; }
};
struct MaxOp {
    static __device__ __forceinline__ double f(double a, double b) { return a > b ? a : b; }
};

// Fixed-order block reduction of one value: butterfly inside each wave64,
// then the four wave results in order.  Every thread must call it.
template <typename Op>
__device__ __forceinline__ double block_reduce(double v, double *sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v = Op::f(v, __shfl_xor(v, off, 64));
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0)
        sh[wave] = v;
    __syncthreads();
    double r = sh[0];
#pragma unroll
    for (int w = 1; w < kBlock / 64; ++w)
        r = Op::f(r, sh[w]);
    return r;
}

// Read-out of node (x, y): post-stream density (FP64, with its residual)
// and velocity (Eqs. 16-17 after the boundary override).
template <typename T, int BCX, int BCY>
__device__ __forceinline__ void readout_node(const char *src, const Layout &lay, const char *med,
                                             const MLayout &mlay, const Geom &g,
                                             const Physics &ph, float s, float inv_s, int y,
                                             uint32_t x, double &rp, float &ux, float &uy)
{
    const Rows R = rows_of<BCY>(src, lay, g, y);
    const Med md{med_row(med, mlay, y), mlay.slot, 2 * mlay.slot};
    float d[9], inc, r;
    const float rho = post_stream<T, BCX>(R, lay, md, g, ph, s, inv_s, x, d, inc, r);
    float jx, jy, Fx, Fy;
    momentum(d, jx, jy);
    if (Elem<T>::kScaled) {
        jx *= inv_s;
        jy *= inv_s;
    }
    velocity(ph, rho, jx, jy, md.eps(x), md.drag(x), md.kn0(x), ux, uy, Fx, Fy);
    rp = (double)rho + (double)r;
}

template <typename T, int BCX, int BCY>
__global__ __launch_bounds__(kBlock) void macro_kernel(const char *src, Layout lay,
                                                        const char *med, MLayout mlay, Geom g,
                                                        Physics ph, float s, float inv_s, int bpr,
                                                        float *rho_out, float *ux_out,
                                                        float *uy_out, float *ux_prev,
                                                        float *uy_prev, double *partials)
{
    __shared__ double sh[kBlock / 64];
    const Node nd = node_of(bpr);
    double v[MAC_SLOTS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (nd.x < (uint32_t)g.nx) {
        double rp;
        float ux, uy;
        readout_node<T, BCX, BCY>(src, lay, med, mlay, g, ph, s, inv_s, nd.y, nd.x, rp, ux, uy);
        const uint32_t o = (uint32_t)nd.y * (uint32_t)g.nx + nd.x;
        if (rho_out)
            rho_out[o] = (float)rp;
        if (ux_out)
            ux_out[o] = ux;
        if (uy_out)
            uy_out[o] = uy;
        v[MAC_FLUX] = rp * (double)ux;
        v[MAC_UX] = ux;
        v[MAC_U2] = (double)ux * ux + (double)uy * uy;
        v[MAC_RHO] = rp;
        v[MAC_QOUT] = (nd.x == (uint32_t)g.nx - 1) ? rp * (double)ux : 0.0;
        if (ux_prev) {
            const uint32_t c = (uint32_t)nd.y * (uint32_t)g.pitch + nd.x;
            const double dx = (double)ux - ux_prev[c], dy = (double)uy - uy_prev[c];
            v[MAC_DU2] = dx * dx + dy * dy;
            ux_prev[c] = ux;
            uy_prev[c] = uy;
        }
    }
#pragma unroll
    for (int k = 0; k < MAC_SLOTS; ++k) {
        const double rr = block_reduce<SumOp>(v[k], sh);
        if (threadIdx.x == 0)
            partials[(int64_t)k * gridDim.x + nd.L] = rr;
    }
}

// The read-out sums of macro_kernel (no field outputs, no residual) with a
// fixed grid: workgroup b walks the lattice's 256-node blocks b, b + G, ...
// and writes one partial per slot, partials[k][b], so the partial count is
// the grid size whatever the lattice size.
template <typename T, int BCX, int BCY>
__global__ __launch_bounds__(kBlock) void macro_strided_kernel(const char *src, Layout lay,
                                                                const char *med, MLayout mlay,
                                                                Geom g, Physics ph, float s,
                                                                float inv_s, int bpr, int nblocks,
                                                                double *partials)
{
    __shared__ double sh[kBlock / 64];
    double v[MAC_SLOTS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int L = blockIdx.x; L < nblocks; L += gridDim.x) {
        const int y = L / bpr;
        const uint32_t x = (uint32_t)(L - y * bpr) * kBlock + threadIdx.x;
        if (x < (uint32_t)g.nx) {
            double rp;
            float ux, uy;
            readout_node<T, BCX, BCY>(src, lay, med, mlay, g, ph, s, inv_s, y, x, rp, ux, uy);
            v[MAC_FLUX] += rp * (double)ux;
            v[MAC_UX] += ux;
            v[MAC_U2] += (double)ux * ux + (double)uy * uy;
            v[MAC_RHO] += rp;
            v[MAC_QOUT] += (x == (uint32_t)g.nx - 1) ? rp * (double)ux : 0.0;
        }
    }
#pragma unroll
    for (int k = 0; k < MAC_SLOTS; ++k) {
        const double rr = block_reduce<SumOp>(v[k], sh);
        if (threadIdx.x == 0)
            partials[(int64_t)k * gridDim.x + blockIdx.x] = rr;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void state_sums_kernel(const char *src, Layout lay, Geom g,
                                                             float inv_s, double *partials,
                                                             int bpr)
{
    __shared__ double sh[kBlock / 64];
    const Node nd = node_of(bpr);
    double mass = 0.0, hmax = 0.0, bad = 0.0;
    if (nd.x < (uint32_t)g.nx) {
        const Rsrc row = state_row<T>(src, lay, nd.y);
        const float rho = ld_f32(row, nd.x * 4, 0);
        double hsum = 0.0;
        bad += isfinite(rho) ? 0.0 : 1.0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const float v = Elem<T>::ld(row, nd.x * sizeof(T), lay.h_off + i * lay.h_slot) * inv_s;
            hsum += (double)v;
            const double a = fabs((double)v);
            hmax = a > hmax ? a : hmax;
            bad += isfinite(v) ? 0.0 : 1.0;
        }
        mass = (double)rho + hsum;
    }
    double r = block_reduce<SumOp>(mass, sh);
    if (threadIdx.x == 0)
        partials[(int64_t)ST_MASS * gridDim.x + nd.L] = r;
    r = block_reduce<MaxOp>(hmax, sh);
    if (threadIdx.x == 0)
        partials[(int64_t)ST_HMAX * gridDim.x + nd.L] = r;
    r = block_reduce<SumOp>(bad, sh);
    if (threadIdx.x == 0)
        partials[(int64_t)ST_BAD * gridDim.x + nd.L] = r;
}

// Read-out of every sample of a batch: per-tile FP64 partials
// [MAC_SLOTS][ntiles] (tiles of kBlock nodes), reduced per sample by
// batch_finish_kernel in a fixed order.
template <typename T, int BCX, int BCY>
__global__ __launch_bounds__(kBlock) void batch_macro_kernel(const SampleDesc *samples,
                                                              const int *tile_sample, int ntiles,
                                                              int parity, double *partials)
{
    __shared__ double sh[kBlock / 64];
    const int t = blockIdx.x;
    const int si = tile_sample[t];
    const SampleDesc &sd = samples[si];
    const int rel = t - sd.tile0;
    const int y = rel / sd.tpr;
    const uint32_t x = (uint32_t)(rel - y * sd.tpr) * kBlock + threadIdx.x;
    double v[MAC_SLOTS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (x < (uint32_t)sd.g.nx) {
        const Rows R = rows_of<BCY>(sd.state[parity], sd.lay, sd.g, y);
        const Med md{med_row(sd.med, sd.mlay, y), sd.mlay.slot, 2 * sd.mlay.slot};
        float d[9], inc, r;
        const float rho =
            post_stream<T, BCX>(R, sd.lay, md, sd.g, sd.ph, sd.s, sd.inv_s, x, d, inc, r);
        float jx, jy, ux, uy, Fx, Fy;
        momentum(d, jx, jy);
        if (Elem<T>::kScaled) {
            jx *= sd.inv_s;
            jy *= sd.inv_s;
        }
        velocity(sd.ph, rho, jx, jy, md.eps(x), md.drag(x), md.kn0(x), ux, uy, Fx, Fy);
        const double rp = (double)rho + (double)r;
        v[MAC_FLUX] = rp * (double)ux;
        v[MAC_UX] = ux;
        v[MAC_U2] = (double)ux * ux + (double)uy * uy;
        v[MAC_RHO] = rp;
        v[MAC_QOUT] = (x == (uint32_t)sd.g.nx - 1) ? rp * (double)ux : 0.0;
    }
#pragma unroll
    for (int k = 0; k < MAC_SLOTS; ++k) {
        const double rr = block_reduce<SumOp>(v[k], sh);
        if (threadIdx.x == 0)
            partials[(int64_t)k * ntiles + t] = rr;
    }
}

// out[s][k] = sum of partials[k][tile0(s) .. tile0(s) + tiles(s)) in order.
__global__ __launch_bounds__(kBlock) void batch_finish_kernel(const SampleDesc *samples,
                                                               const double *partials, int slots,
                                                               int ntiles, double *out)
{
    __shared__ double sh[kBlock / 64];
    const SampleDesc &sd = samples[blockIdx.x];
    const int t0 = sd.tile0, n = sd.tpr * sd.g.ny;
    for (int k = 0; k < slots; ++k) {
        const double *p = partials + (int64_t)k * ntiles + t0;
        double v = 0.0;
        for (int j = threadIdx.x; j < n; j += kBlock)
            v += p[j];
        const double r = block_reduce<SumOp>(v, sh);
        if (threadIdx.x == 0)
            out[(int64_t)blockIdx.x * slots + k] = r;
    }
}

__global__ __launch_bounds__(kBlock) void finish_kernel(const double *partials, int slots,
                                                         int blocks, unsigned max_mask,
                                                         double *out)
{
    __shared__ double sh[kBlock / 64];
    for (int k = 0; k < slots; ++k) {
        const bool is_max = (max_mask >> k) & 1u;
        const double *p = partials + (int64_t)k * blocks;
        double v = 0.0;
        for (int j = threadIdx.x; j < blocks; j += kBlock)
            v = is_max ? (p[j] > v ? p[j] : v) : v + p[j];
        const double r = is_max ? block_reduce<MaxOp>(v, sh) : block_reduce<SumOp>(v, sh);
        if (threadIdx.x == 0)
            out[k] = r;
    }
}

// ---------------------------------------------------------------- set-up

__global__ __launch_bounds__(kBlock) void fields_kernel(char *med, MLayout mlay, Geom g,
                                                         double nu, double *partials, int bpr)
{
    __shared__ double sh[kBlock / 64];
    const Node nd = node_of(bpr);
    double bad = 0.0;
    if (nd.x < (uint32_t)g.nx) {
        const Rsrc row = med_row(med, mlay, nd.y);
        const float e = ld_f32(row, nd.x * 4, 0), k = ld_f32(row, nd.x * 4, mlay.slot),
                    kn = ld_f32(row, nd.x * 4, 2 * mlay.slot);
        const bool ok = (e >= 0.0f && e <= 1.0f) && (k > 0.0f) && (kn >= 0.0f) && isfinite(kn);
        bad = ok ? 0.0 : 1.0;
        double d = 0.0;
        if (ok && e > 0.0f && isfinite(k))
            d = (double)e * nu / (double)k;
        st_f32(row, nd.x * 4, mlay.slot, (float)d, false);
    }
    const double r = block_reduce<SumOp>(bad, sh);
    if (threadIdx.x == 0)
        partials[(int64_t)FLD_BAD * gridDim.x + nd.L] = r;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void init_state_kernel(char *dst, Layout lay, Geom g,
                                                             int ramp, double rho0,
                                                             double rho_in, double rho_out,
                                                             float s, int bpr)
{
    const Node nd = node_of(bpr);
    if (nd.x >= (uint32_t)g.nx)
        return;
    double rho = rho0;
    if (ramp)
        rho = g.nx > 1 ? rho_in + (rho_out - rho_in) * (double)nd.x / (double)(g.nx - 1)
                       : rho_in;
    const float hi = (float)rho;
    const float lo = (float)(rho - (double)hi);
    const Rsrc row = state_row<T>(dst, lay, nd.y);
    st_f32(row, nd.x * 4, 0, hi, false);
#pragma unroll
    for (int i = 0; i < 9; ++i)
        Elem<T>::st(row, nd.x * sizeof(T), lay.h_off + i * lay.h_slot, w_of(i) * lo * s);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void populations_kernel(const char *src, Layout lay,
                                                              Geom g, float inv_s, double *out,
                                                              int bpr)
{
    const Node nd = node_of(bpr);
    if (nd.x >= (uint32_t)g.nx)
        return;
    const Rsrc row = state_row<T>(src, lay, nd.y);
    const double rho = ld_f32(row, nd.x * 4, 0);
    const int64_t n = (int64_t)g.nx * g.ny;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double w = i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
        const float h = Elem<T>::ld(row, nd.x * sizeof(T), lay.h_off + i * lay.h_slot) * inv_s;
        out[i * n + (int64_t)nd.y * g.nx + nd.x] = w * rho + (double)h;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void rescale_kernel(char *st, Layout lay, Geom g, float f,
                                                          int bpr)
{
    const Node nd = node_of(bpr);
    if (nd.x >= (uint32_t)g.nx)
        return;
    const Rsrc row = state_row<T>(st, lay, nd.y);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const uint32_t so = lay.h_off + i * lay.h_slot;
        Elem<T>::st(row, nd.x * sizeof(T), so, Elem<T>::ld(row, nd.x * sizeof(T), so) * f);
    }
}

// ------------------------------------------------------------- launchers

template <typename T, int BCX, int BCY>
static hipError_t sweep_t(const char *src, char *dst, const Layout &lay, const char *med,
                          const MLayout &mlay, const Geom &g, const Physics &ph, float s,
                          float inv_s, float *hist, hipStream_t st)
{
    const Launch l = launch_of(g);
    if (hist)
        hipLaunchKernelGGL((sweep_kernel<T, BCX, BCY, true>), dim3(l.blocks), dim3(kBlock), 0,
                           st, src, dst, lay, med, mlay, g, ph, s, inv_s, hist,
                           l.blocks_per_row);
    else
        hipLaunchKernelGGL((sweep_kernel<T, BCX, BCY, false>), dim3(l.blocks), dim3(kBlock), 0,
                           st, src, dst, lay, med, mlay, g, ph, s, inv_s, hist,
                           l.blocks_per_row);
    return hipGetLastError();
}

template <typename T, int BCX, int BCY>
static hipError_t sweep2_t(const char *src, char *dst, const Layout &lay, const char *med,
                           const MLayout &mlay, const Geom &g, const Physics &ph, float s,
                           float inv_s, int band, float *hist1, float *hist2, hipStream_t st)
{
    if (band < 1 || (hist1 == nullptr) != (hist2 == nullptr))
        return hipErrorInvalidValue;
    const int nstrips = (g.nx + kStrip2 - 1) / kStrip2;
    const int groups = (nstrips + kBlock / 64 - 1) / (kBlock / 64);
    const int64_t blocks = (int64_t)groups * ((g.ny + band - 1) / band);
    if (blocks > 0x7fffffff)
        return hipErrorInvalidValue;
    if (hist1)
        hipLaunchKernelGGL((sweep2_kernel<T, BCX, BCY, true>), dim3((unsigned)blocks),
                           dim3(kBlock), 0, st, src, dst, lay, med, mlay, g, ph, s, inv_s, band,
                           groups, hist1, hist2);
    else
        hipLaunchKernelGGL((sweep2_kernel<T, BCX, BCY, false>), dim3((unsigned)blocks),
                           dim3(kBlock), 0, st, src, dst, lay, med, mlay, g, ph, s, inv_s, band,
                           groups, hist1, hist2);
    return hipGetLastError();
}

template <typename T, int BCX, int BCY>
static hipError_t sweep3x_t(const char *src, char *dst, const Layout &lay, const char *med,
                            const MLayout &mlay, const Geom &g, const Physics &ph, float s,
                            float inv_s, int band, float *hist1, float *hist2, float *hist3,
                            hipStream_t st)
{
    const bool hist = hist1 != nullptr;
    if (band < 1 || (hist2 != nullptr) != hist || (hist3 != nullptr) != hist)
        return hipErrorInvalidValue;
    const int nstrips = (g.nx + kStrip3 - 1) / kStrip3;
    const int groups = (nstrips + kBlock / 64 - 1) / (kBlock / 64);
    const int64_t blocks = (int64_t)groups * ((g.ny + band - 1) / band);
    if (blocks > 0x7fffffff)
        return hipErrorInvalidValue;
    if (hist)
        hipLaunchKernelGGL((sweep3x_kernel<T, BCX, BCY, true>), dim3((unsigned)blocks),
                           dim3(kBlock), 0, st, src, dst, lay, med, mlay, g, ph, s, inv_s, band,
                           groups, hist1, hist2, hist3);
    else
        hipLaunchKernelGGL((sweep3x_kernel<T, BCX, BCY, false>), dim3((unsigned)blocks),
                           dim3(kBlock), 0, st, src, dst, lay, med, mlay, g, ph, s, inv_s, band,
                           groups, hist1, hist2, hist3);
    return hipGetLastError();
}

template <typename T, int BCX, int BCY>
static hipError_t macro_t(const char *src, const Layout &lay, const char *med,
                          const MLayout &mlay, const Geom &g, const Physics &ph, float s,
                          float inv_s,
                          float *rho_out, float *ux_out, float *uy_out, float *ux_prev,
                          float *uy_prev, double *partials, hipStream_t st)
{
    const Launch l = launch_of(g);
    hipLaunchKernelGGL((macro_kernel<T, BCX, BCY>), dim3(l.blocks), dim3(kBlock), 0, st, src,
                       lay, med, mlay, g, ph, s, inv_s, l.blocks_per_row, rho_out, ux_out,
                       uy_out, ux_prev, uy_prev, partials);
    return hipGetLastError();
}

template <typename T, int BCX, int BCY>
static hipError_t macro_strided_t(const char *src, const Layout &lay, const char *med,
                                  const MLayout &mlay, const Geom &g, const Physics &ph, float s,
                                  float inv_s, int grid, double *partials, hipStream_t st)
{
    const Launch l = launch_of(g);
    hipLaunchKernelGGL((macro_strided_kernel<T, BCX, BCY>), dim3(grid), dim3(kBlock), 0, st, src,
                       lay, med, mlay, g, ph, s, inv_s, l.blocks_per_row, l.blocks, partials);
    return hipGetLastError();
}

// Dispatch a (storage, bc_x, bc_y) triple to a template instance.
#define LBK_DISPATCH_BC(FN, T, ...)                                                          \
    switch (bcx * 2 + bcy) {                                                                 \
    case 0: return FN<T, BC_PERIODIC, BC_PERIODIC>(__VA_ARGS__);                             \
    case 1: return FN<T, BC_PERIODIC, BC_WALL>(__VA_ARGS__);                                 \
    case 2: return FN<T, BC_WALL, BC_PERIODIC>(__VA_ARGS__);                                 \
    case 3: return FN<T, BC_WALL, BC_WALL>(__VA_ARGS__);                                     \
    case 4: return FN<T, BC_PRESSURE, BC_PERIODIC>(__VA_ARGS__);                             \
    case 5: return FN<T, BC_PRESSURE, BC_WALL>(__VA_ARGS__);                                 \
    default: return hipErrorInvalidValue;                                                    \
    }

#define LBK_DISPATCH(FN, ...)                                                                \
    switch (storage) {                                                                       \
    case 0: LBK_DISPATCH_BC(FN, float, __VA_ARGS__)                                          \
    case 1: LBK_DISPATCH_BC(FN, __half, __VA_ARGS__)                                         \
    case 2: LBK_DISPATCH_BC(FN, __hip_bfloat16, __VA_ARGS__)                                 \
    default: return hipErrorInvalidValue;                                                    \
    }

// Launch KERNEL<T> for the storage type over the lattice grid; the kernel's
// last parameter is the blocks-per-row count.
#define LBK_LAUNCH_T(KERNEL, ...)                                                            \
    do {                                                                                     \
        const Launch l = launch_of(g);                                                       \
        switch (storage) {                                                                   \
        case 0:                                                                              \
            hipLaunchKernelGGL(KERNEL<float>, dim3(l.blocks), dim3(kBlock), 0, st,           \
                               __VA_ARGS__, l.blocks_per_row);                              \
            break;                                                                           \
        case 1:                                                                              \
            hipLaunchKernelGGL(KERNEL<__half>, dim3(l.blocks), dim3(kBlock), 0, st,          \
                               __VA_ARGS__, l.blocks_per_row);                              \
            break;                                                                           \
        case 2:                                                                              \
            hipLaunchKernelGGL(KERNEL<__hip_bfloat16>, dim3(l.blocks), dim3(kBlock), 0, st,  \
                               __VA_ARGS__, l.blocks_per_row);                              \
            break;                                                                           \
        default:                                                                             \
            return hipErrorInvalidValue;                                                     \
        }                                                                                    \
    } while (0)

hipError_t launch_sweep(int storage, int bcx, int bcy, const char *src, char *dst,
                        const Layout &lay, const char *med, const MLayout &mlay, const Geom &g,
                        const Physics &ph, float s, float inv_s, float *hist, hipStream_t st)
{
    if (bcy < 0 || bcy > 1)
        return hipErrorInvalidValue;
    LBK_DISPATCH(sweep_t, src, dst, lay, med, mlay, g, ph, s, inv_s, hist, st)
}

hipError_t launch_sweep2(int storage, int bcx, int bcy, const char *src, char *dst,
                         const Layout &lay, const char *med, const MLayout &mlay, const Geom &g,
                         const Physics &ph, float s, float inv_s, int band, float *hist1,
                         float *hist2, hipStream_t st)
{
    if (bcy < 0 || bcy > 1)
        return hipErrorInvalidValue;
    LBK_DISPATCH(sweep2_t, src, dst, lay, med, mlay, g, ph, s, inv_s, band, hist1, hist2, st)
}

hipError_t launch_sweep3x(int storage, int bcx, int bcy, const char *src, char *dst,
                          const Layout &lay, const char *med, const MLayout &mlay, const Geom &g,
                          const Physics &ph, float s, float inv_s, int band, float *hist1,
                          float *hist2, float *hist3, hipStream_t st)
{
    if (bcy < 0 || bcy > 1)
        return hipErrorInvalidValue;
    LBK_DISPATCH(sweep3x_t, src, dst, lay, med, mlay, g, ph, s, inv_s, band, hist1, hist2, hist3,
                 st)
}

hipError_t launch_macro(int storage, int bcx, int bcy, const char *src, const Layout &lay,
                        const char *med, const MLayout &mlay, const Geom &g, const Physics &ph,
                        float s, float inv_s, float *rho_out, float *ux_out, float *uy_out,
                        float *ux_prev, float *uy_prev, double *partials, hipStream_t st)
{
    if (bcy < 0 || bcy > 1)
        return hipErrorInvalidValue;
    LBK_DISPATCH(macro_t, src, lay, med, mlay, g, ph, s, inv_s, rho_out, ux_out, uy_out,
                 ux_prev, uy_prev, partials, st)
}

hipError_t launch_macro_strided(int storage, int bcx, int bcy, const char *src,
                                const Layout &lay, const char *med, const MLayout &mlay,
                                const Geom &g, const Physics &ph, float s, float inv_s, int grid,
                                double *partials, hipStream_t st)
{
    if (bcy < 0 || bcy > 1 || grid < 1)
        return hipErrorInvalidValue;
    LBK_DISPATCH(macro_strided_t, src, lay, med, mlay, g, ph, s, inv_s, grid, partials, st)
}

hipError_t launch_state_sums(int storage, const char *src, const Layout &lay, const Geom &g,
                             float inv_s, double *partials, hipStream_t st)
{
    LBK_LAUNCH_T(state_sums_kernel, src, lay, g, inv_s, partials);
    return hipGetLastError();
}

hipError_t launch_finish(const double *partials, int slots, int blocks, unsigned max_mask,
                         double *out, hipStream_t st)
{
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(kBlock), 0, st, partials, slots, blocks,
                       max_mask, out);
    return hipGetLastError();
}

hipError_t launch_fields(char *med, const MLayout &mlay, const Geom &g, double nu,
                         double *partials, hipStream_t st)
{
    const Launch l = launch_of(g);
    hipLaunchKernelGGL(fields_kernel, dim3(l.blocks), dim3(kBlock), 0, st, med, mlay, g, nu,
                       partials, l.blocks_per_row);
    return hipGetLastError();
}

hipError_t launch_init_state(int storage, char *dst, const Layout &lay, const Geom &g, int ramp,
                             double rho0, double rho_in, double rho_out, float s,
                             hipStream_t st)
{
    LBK_LAUNCH_T(init_state_kernel, dst, lay, g, ramp, rho0, rho_in, rho_out, s);
    return hipGetLastError();
}

hipError_t launch_populations(int storage, const char *src, const Layout &lay, const Geom &g,
                              float inv_s, double *out, hipStream_t st)
{
    LBK_LAUNCH_T(populations_kernel, src, lay, g, inv_s, out);
    return hipGetLastError();
}

hipError_t launch_rescale(int storage, char *state, const Layout &lay, const Geom &g, int k,
                          hipStream_t st)
{
    const float f = ldexpf(1.0f, k);
    LBK_LAUNCH_T(rescale_kernel, state, lay, g, f);
    return hipGetLastError();
}

// ---------------------------------------------------------- batch launch

template <typename T, int BCX, int BCY>
static hipError_t batch_sweep_t(const SampleDesc *samples, const int *tile_sample, int ntiles,
                                int parity, int tile_x, int rows, int grid, hipStream_t st)
{
    if (grid > 0)
        hipLaunchKernelGGL((batch_sweep_kernel<T, BCX, BCY, true>), dim3(grid), dim3(tile_x), 0,
                           st, samples, tile_sample, ntiles, rows, parity);
    else
        hipLaunchKernelGGL((batch_sweep_kernel<T, BCX, BCY, false>), dim3(ntiles), dim3(tile_x),
                           0, st, samples, tile_sample, ntiles, rows, parity);
    return hipGetLastError();
}

template <typename T, int BCX, int BCY>
static hipError_t batch_macro_t(const SampleDesc *samples, const int *tile_sample, int ntiles,
                                int parity, double *partials, hipStream_t st)
{
    hipLaunchKernelGGL((batch_macro_kernel<T, BCX, BCY>), dim3(ntiles), dim3(kBlock), 0, st,
                       samples, tile_sample, ntiles, parity, partials);
    return hipGetLastError();
}

hipError_t launch_batch_sweep(int storage, int bcx, int bcy, const SampleDesc *samples,
                              const int *tile_sample, int ntiles, int parity, int tile_x,
                              int rows, int grid, hipStream_t st)
{
    if (bcy < 0 || bcy > 1 || tile_x < 64 || tile_x > kBatchMaxTile || (tile_x & 63) ||
        rows < 1 || grid < 0 || ntiles < 0)
        return hipErrorInvalidValue;
    if (ntiles == 0)
        return hipSuccess;
    LBK_DISPATCH(batch_sweep_t, samples, tile_sample, ntiles, parity, tile_x, rows, grid, st)
}

template <typename T, int BCX, int BCY>
static hipError_t batch_rec_sweep2_t(const AdjSampleDesc *samples, const int *tile_sample,
                                     int ntiles, int band, LevelSel src, LevelSel dst,
                                     int hist_slot, hipStream_t st)
{
    if (hist_slot >= 0)
        hipLaunchKernelGGL((batch_rec_sweep2_kernel<T, BCX, BCY, true>), dim3(ntiles),
                           dim3(kBlock), 0, st, samples, tile_sample, band, src, dst, hist_slot);
    else
        hipLaunchKernelGGL((batch_rec_sweep2_kernel<T, BCX, BCY, false>), dim3(ntiles),
                           dim3(kBlock), 0, st, samples, tile_sample, band, src, dst, hist_slot);
    return hipGetLastError();
}

hipError_t launch_batch_rec_sweep2(int storage, int bcx, int bcy, const AdjSampleDesc *samples,
                                   const int *tile_sample, int ntiles, int band, LevelSel src,
                                   LevelSel dst, int hist_slot, hipStream_t st)
{
    if (bcy < 0 || bcy > 1 || band < 1 || ntiles < 0)
        return hipErrorInvalidValue;
    if (ntiles == 0)
        return hipSuccess;
    LBK_DISPATCH(batch_rec_sweep2_t, samples, tile_sample, ntiles, band, src, dst, hist_slot, st)
}

template <typename T, int BCX, int BCY>
static hipError_t batch_sweep2_t(const SampleDesc *samples, const int *tile_sample, int ntiles,
                                 int parity, int band, hipStream_t st)
{
    hipLaunchKernelGGL((batch_sweep2_kernel<T, BCX, BCY>), dim3(ntiles), dim3(kBlock), 0, st,
                       samples, tile_sample, band, parity);
    return hipGetLastError();
}

hipError_t launch_batch_sweep2(int storage, int bcx, int bcy, const SampleDesc *samples,
                               const int *tile_sample, int ntiles, int parity, int band,
                               hipStream_t st)
{
    if (bcy < 0 || bcy > 1 || band < 1 || ntiles < 0)
        return hipErrorInvalidValue;
    if (ntiles == 0)
        return hipSuccess;
    LBK_DISPATCH(batch_sweep2_t, samples, tile_sample, ntiles, parity, band, st)
}

hipError_t launch_batch_macro(int storage, int bcx, int bcy, const SampleDesc *samples,
                              const int *tile_sample, int ntiles, int parity, double *partials,
                              hipStream_t st)
{
    if (bcy < 0 || bcy > 1)
        return hipErrorInvalidValue;
    LBK_DISPATCH(batch_macro_t, samples, tile_sample, ntiles, parity, partials, st)
}

hipError_t launch_batch_finish(const SampleDesc *samples, int nsamples, const double *partials,
                               int slots, int ntiles, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(batch_finish_kernel, dim3(nsamples), dim3(kBlock), 0, st, samples,
                       partials, slots, ntiles, out);
    return hipGetLastError();
}

template <typename T, int BCX, int BCY>
static hipError_t batch_rec_t(const AdjSampleDesc *samples, const int *tile_sample, int ntiles,
                              int tile_x, int rows, LevelSel src, LevelSel dst, int hist_slot,
                              hipStream_t st)
{
    if (hist_slot >= 0)
        hipLaunchKernelGGL((batch_rec_sweep_kernel<T, BCX, BCY, true>), dim3(ntiles),
                           dim3(tile_x), 0, st, samples, tile_sample, ntiles, rows, src, dst,
                           hist_slot);
    else
        hipLaunchKernelGGL((batch_rec_sweep_kernel<T, BCX, BCY, false>), dim3(ntiles),
                           dim3(tile_x), 0, st, samples, tile_sample, ntiles, rows, src, dst,
                           hist_slot);
    return hipGetLastError();
}

hipError_t launch_batch_rec_sweep(int storage, int bcx, int bcy, const AdjSampleDesc *samples,
                                  const int *tile_sample, int ntiles, int tile_x, int rows,
                                  LevelSel src, LevelSel dst, int hist_slot, hipStream_t st)
{
    if (bcy < 0 || bcy > 1 || tile_x < 64 || tile_x > kBatchMaxTile || (tile_x & 63) ||
        rows < 1 || ntiles < 0 || src.region < 0 || src.region > 3 || dst.region < 0 ||
        dst.region > 3)
        return hipErrorInvalidValue;
    if (ntiles == 0)
        return hipSuccess;
    LBK_DISPATCH(batch_rec_t, samples, tile_sample, ntiles, tile_x, rows, src, dst, hist_slot, st)
}

} // namespace lbk
