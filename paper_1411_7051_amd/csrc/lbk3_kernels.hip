// lbk3_kernels.hip -- the D3Q19 form of the fused sweep: the same model
// (Eqs. 12, 14-17 with Eqs. 2-8: Guo's porous equilibrium and forcing, the
// local Knudsen number, the selected slip correlation, Eq. 17 or the
// Forchheimer quadratic, bounce-back, pressure planes) on nineteen
// velocities: rest, the six axis links (weight 1/18) and the twelve face
// diagonals (1/36), cs^2 = 1/3.
//
// Storage is the density split of the D2Q9 path: per node an FP32 density
// and nineteen deviations h_i = f*_i - w_i rho in the storage type, in row
// blocks [rho | h_0 .. h_18] of `pitch` elements per slot; a row is one
// (y, z) line of x, row index z * ny + y.  A node pulls from the nine rows
// (y + a, z + b), a, b in {-1, 0, 1}.  One node per thread, 256 threads per
// block along x, grid remapped into XCD bands as in the D2Q9 sweep.
#include "lbk3_kernels.h"

namespace lbk {

namespace {

// D3Q19, pairs (i, i + 1) opposite for odd i.
__host__ __device__ constexpr int ex3(int i)
{
    constexpr int t[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return t[i];
}
__host__ __device__ constexpr int ey3(int i)
{
    constexpr int t[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return t[i];
}
__host__ __device__ constexpr int ez3(int i)
{
    constexpr int t[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return t[i];
}
__host__ __device__ constexpr int opp3(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr float w3(int i)
{
    return i == 0 ? 1.0f / 3.0f : (i <= 6 ? 1.0f / 18.0f : 1.0f / 36.0f);
}

// Fixed-order block reductions (wave shuffles, then the waves in order).
__device__ __forceinline__ double block_red(double v, double *sh, bool is_max)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off, 64);
        v = is_max ? (o > v ? o : v) : v + o;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0)
        sh[wave] = v;
    __syncthreads();
    double r = sh[0];
#pragma unroll
    for (int w = 1; w < kBlock3 / 64; ++w)
        r = is_max ? (sh[w] > r ? sh[w] : r) : r + sh[w];
    return r;
}
__device__ __forceinline__ double block_sum(double v, double *sh) { return block_red(v, sh, false); }
__device__ __forceinline__ double block_max(double v, double *sh) { return block_red(v, sh, true); }

__device__ __forceinline__ int xcd_remap3(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int j = b & 7, idx = b >> 3;
    return j * q + (j < r ? j : r) + idx;
}

// Cache policy of the D3Q19 population loads: default (cached).  A node
// pulls from nine rows, three of them a whole z-plane of rows away in the
// launch order; with streaming (nontemporal) population loads those rows'
// density lines were evicted before their reuse and fetched again (114
// against 100 bytes per node fetched from HBM at FP32 on the 256^3 sphere
// medium, 3% slower).  The two-dimensional sweep keeps nontemporal loads.
constexpr int kAux3 = 0;

struct Node3 {
    int y, z;
    uint32_t x;
};

__device__ __forceinline__ Node3 node3_of(const Geom3 &g, int bpr)
{
    const int L = xcd_remap3(blockIdx.x, gridDim.x);
    const int row = L / bpr;
    Node3 n;
    n.z = row / g.ny;
    n.y = row - n.z * g.ny;
    n.x = (uint32_t)(L - row * bpr) * kBlock3 + threadIdx.x;
    return n;
}

__device__ __forceinline__ uint64_t row3(const Geom3 &g, int y, int z)
{
    return (uint64_t)z * g.ny + y;
}

// The nine rows a node pulls from; r[a][b] is row (y + a - 1, z + b - 1).
// A row beyond a wall is replaced by the node's own row (entries unused).
struct Rows3 {
    Rsrc r[3][3];
    bool wym, wyp, wzm, wzp;
};

template <int BCY, int BCZ>
__device__ __forceinline__ Rows3 rows3_of(const char *base, const Layout &L, const Geom3 &g,
                                          int y, int z)
{
    Rows3 R;
    int ys[3] = {y - 1, y, y + 1}, zs[3] = {z - 1, z, z + 1};
    R.wym = R.wyp = R.wzm = R.wzp = false;
    if (BCY == BC_PERIODIC) {
        ys[0] = y == 0 ? g.ny - 1 : ys[0];
        ys[2] = y == g.ny - 1 ? 0 : ys[2];
    } else {
        // the row is the workgroup's: scalar wall flags keep the selects
        // of buffer resources scalar
        R.wym = __builtin_amdgcn_readfirstlane(y == 0 ? 1 : 0) != 0;
        R.wyp = __builtin_amdgcn_readfirstlane(y == g.ny - 1 ? 1 : 0) != 0;
        ys[0] = R.wym ? y : ys[0];
        ys[2] = R.wyp ? y : ys[2];
    }
    if (BCZ == BC_PERIODIC) {
        zs[0] = z == 0 ? g.nz - 1 : zs[0];
        zs[2] = z == g.nz - 1 ? 0 : zs[2];
    } else {
        R.wzm = __builtin_amdgcn_readfirstlane(z == 0 ? 1 : 0) != 0;
        R.wzp = __builtin_amdgcn_readfirstlane(z == g.nz - 1 ? 1 : 0) != 0;
        zs[0] = R.wzm ? z : zs[0];
        zs[2] = R.wzp ? z : zs[2];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            R.r[a][b] = make_rsrc(base + row3(g, ys[a], zs[b]) * L.row, (uint32_t)L.row);
    return R;
}

// Pull of node (x, y, z): d_i = f_i - w_i rc in the storage unit; a link
// crossing a wall returns the node's own opposite deviation.
template <typename T, int BCX>
__device__ __forceinline__ void pull3(const Rows3 &R, const Layout &L, const Geom3 &g, float s,
                                      uint32_t x, float &rc, float (&d)[19])
{
    uint32_t xm = x - 1, xp = x + 1;
    bool wxm = false, wxp = false;
    if (BCX == BC_PERIODIC) {
        xm = (x == 0) ? (uint32_t)g.nx - 1 : xm;
        xp = (x == (uint32_t)g.nx - 1) ? 0 : xp;
    } else if (BCX == BC_WALL) {
        wxm = (x == 0);
        wxp = (x == (uint32_t)g.nx - 1);
        xm = wxm ? x : xm;
        xp = wxp ? x : xp;
    }
    constexpr uint32_t es = sizeof(T);
    const Rsrc &own = R.r[1][1];
    rc = ld_f32(own, x * 4, 0);
    d[0] = Elem<T>::template ld<kAux3>(own, x * es, L.h_off);
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        const int ex = ex3(i), ey = ey3(i), ez = ez3(i);
        const uint32_t sx = ex == 1 ? xm : (ex == -1 ? xp : x);
        const bool wall = (ey == 1 && R.wym) || (ey == -1 && R.wyp) || (ez == 1 && R.wzm) ||
                          (ez == -1 && R.wzp); // uniform
        const float ws = Elem<T>::kScaled ? w3(i) * s : w3(i);
        if (wall) {
            d[i] = Elem<T>::template ld<kAux3>(own, x * es, L.h_off + opp3(i) * L.h_slot);
        } else {
            const Rsrc &src = R.r[1 - ey][1 - ez];
            const float rn = ld_f32(src, sx * 4, 0);
            const float h = Elem<T>::template ld<kAux3>(src, sx * es, L.h_off + i * L.h_slot);
            d[i] = ws * (rn - rc) + h;
        }
        if (BCX == BC_WALL) {
            const bool wall_x = (ex == 1 && wxm) || (ex == -1 && wxp);
            if (wall_x)
                d[i] = Elem<T>::template ld<kAux3>(own, x * es, L.h_off + opp3(i) * L.h_slot);
        }
    }
}

// rho = FP32(rc + sum d / s), inc = rho - rc, r the exact residual (Fast2Sum).
template <typename T>
__device__ __forceinline__ float density3(float rc, const float (&d)[19], float inv_s,
                                          float &inc, float &r)
{
    float sum = 0.0f;
#pragma unroll
    for (int i = 0; i < 19; ++i)
        sum += d[i];
    const float sp = Elem<T>::kScaled ? sum * inv_s : sum;
    const float rho = rc + sp;
    inc = rho - rc;
    r = sp - inc;
    return rho;
}

// sum_i e_i d_i over the opposite pairs.
__device__ __forceinline__ void momentum3(const float (&d)[19], float (&j)[3])
{
    j[0] = (d[1] - d[2]) + (d[7] - d[8]) + (d[9] - d[10]) + (d[11] - d[12]) + (d[13] - d[14]);
    j[1] = (d[3] - d[4]) + (d[7] - d[8]) + (d[10] - d[9]) + (d[15] - d[16]) + (d[17] - d[18]);
    j[2] = (d[5] - d[6]) + (d[11] - d[12]) + (d[14] - d[13]) + (d[15] - d[16]) + (d[18] - d[17]);
}

// Eq. 16b solved as Eq. 17 (or the Forchheimer quadratic of Eq. 2) with
// k_a = k f_c(Kn), f_c = den / num from the selected correlation; one
// reciprocal gives both u and A u (see the D2Q9 velocity solve).
__device__ __forceinline__ void velocity3(const Physics3 &p3, float rho, const float (&j)[3],
                                          float eps, float drag, float kn0, float (&u)[3],
                                          float (&F)[3])
{
    const Physics &ph = p3.ph;
    const float rinv = __builtin_amdgcn_rcpf(rho);
    const float kn = ph.kn_local ? kn0 * (ph.rho_ref * rinv) : kn0;
    float num, den;
    fc_parts(ph, kn, num, den);
    const float G[3] = {ph.gx, ph.gy, p3.gz};
    float v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        v[a] = j[a] * rinv + 0.5f * eps * G[a];
    float g, ag, B = 0.0f;
    if (ph.feps == 0.0f) {
        const float dn = drag * num;
        const float R2 = 2.0f * __builtin_amdgcn_rcpf(2.0f * den + dn);
        g = den * R2;
        ag = dn * R2;
    } else {
        const float A = drag * num * __builtin_amdgcn_rcpf(den);
        B = ph.feps * __builtin_sqrtf(eps * A * ph.inv_nu);
        const float c0 = 1.0f + 0.5f * A;
        const float wn = __builtin_sqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        g = 2.0f / (c0 + __builtin_sqrtf(c0 * c0 + 2.0f * B * wn));
        ag = A * g;
    }
    const bool solid = !(eps > 0.0f);
#pragma unroll
    for (int a = 0; a < 3; ++a)
        u[a] = solid ? 0.0f : g * v[a];
    const float bu = (ph.feps != 0.0f) ? B * __builtin_sqrtf(u[0] * u[0] + u[1] * u[1] + u[2] * u[2])
                                       : 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        F[a] = solid ? -2.0f * j[a] * rinv : eps * G[a] - ag * v[a] - bu * u[a];
}

// BGK + Guo in deviation form over the opposite pairs (see the D2Q9
// collide): h*_i, h*_opp = (1 - omega) d_i + w_i C + w_i rho (4.5 E / eps +/- 3 P).
template <typename T>
__device__ __forceinline__ void collide3(const Physics &ph, float rho, float inc, float r,
                                         const float (&d)[19], const float (&u)[3],
                                         const float (&F)[3], float eps, float s,
                                         float (&hs)[19])
{
    const bool solid = !(eps > 0.0f);
    const float ie = solid ? 0.0f : __builtin_amdgcn_rcpf(eps);
    const float om = ph.omega, cg = ph.guo, keep = 1.0f - om;
    float C = om * r - keep * inc +
              rho * ie *
                  (-1.5f * om * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) -
                   3.0f * cg * (u[0] * F[0] + u[1] * F[1] + u[2] * F[2]));
    float rs = rho;
    if (Elem<T>::kScaled) {
        C *= s;
        rs *= s;
    }
    const float Kb = 4.5f * rs * ie, Mb = 3.0f * rs;
    hs[0] = keep * d[0] + w3(0) * C;
#pragma unroll
    for (int i = 1; i < 19; i += 2) {
        const float w = w3(i);
        const float eu = edot(ex3(i), ey3(i), ez3(i), u[0], u[1], u[2]);
        const float q = cg * edot(ex3(i), ey3(i), ez3(i), F[0], F[1], F[2]);
        const float P = om * eu + q;
        const float E = eu * (P + q);
        const float X = (w * Kb) * E + w * C;
        const float Y = (w * Mb) * P;
        hs[i] = keep * d[i] + (X + Y);
        hs[i + 1] = keep * d[i + 1] + (X - Y);
    }
}

struct Med3 {
    Rsrc row;
    uint32_t slot, slot2; // byte offsets of the drag and kn0 slots
    __device__ float eps(uint32_t x) const { return ld_f32(row, x * 4, 0); }
    __device__ float drag(uint32_t x) const { return ld_f32(row, x * 4, slot); }
    __device__ float kn0(uint32_t x) const { return ld_f32(row, x * 4, slot2); }
};

// Post-stream deviations of node x (pressure planes: non-equilibrium
// extrapolation from the neighbouring plane, as in the D2Q9 sweep).  A
// pressure-plane node pulls at its neighbour xn with the same code as every
// other lane, so that only the extrapolation itself diverges: with 256-wide
// rows, half the waves hold a boundary lane.
template <typename T, int BCX>
__device__ __forceinline__ float post_stream3(const Rows3 &R, const Layout &L, const Med3 &md,
                                              const Geom3 &g, const Physics3 &p3, float s,
                                              float inv_s, uint32_t x, float (&d)[19],
                                              float &inc, float &r)
{
    const Physics &ph = p3.ph;
    const bool bnode = BCX == BC_PRESSURE && (x == 0 || x == (uint32_t)g.nx - 1);
    const uint32_t xs = !bnode ? x : (x == 0 ? 1u : (uint32_t)g.nx - 2);
    float rc;
    pull3<T, BCX>(R, L, g, s, xs, rc, d);
    const float rho = density3<T>(rc, d, inv_s, inc, r);
    if (BCX == BC_PRESSURE && bnode) {
        // d, rho, inc, r are the neighbour's: f_i = f_eq_i(rho_b, u_n; eps_b)
        // + f_i(n) - f_eq_i(rho_n, u_n; eps_n)
        float j[3], u[3], F[3];
        momentum3(d, j);
        if (Elem<T>::kScaled) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
                j[a] *= inv_s;
        }
        const float en = md.eps(xs), eb = md.eps(x);
        velocity3(p3, rho, j, en, md.drag(xs), md.kn0(xs), u, F);
        const bool in = (x == 0);
        const float rb = in ? ph.rin_hi : ph.rout_hi;
        const float rbl = in ? ph.rin_lo : ph.rout_lo;
        // f_eq_i(rho_b, u; eps_b) - f_eq_i(rho_n, u; eps_n) of Eq. 14 as
        // w_i [a e.u + b (4.5 (e.u)^2 - 1.5 u.u)], each equilibrium's
        // deviation from w_i rho vanishing at eps = 0; the pairs (i, i + 1)
        // are opposite, so e.u is formed once per pair
        const bool sb = !(eb > 0.0f), sn = !(en > 0.0f);
        const float a = 3.0f * ((sb ? 0.0f : rb) - (sn ? 0.0f : rho));
        const float b = (sb ? 0.0f : rb * __builtin_amdgcn_rcpf(eb)) -
                        (sn ? 0.0f : rho * __builtin_amdgcn_rcpf(en));
        const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const float c = (rbl - r) - inc; // w_i (rbl - r) - w_i inc, over w_i
        auto phys = [&](float v) { return Elem<T>::kScaled ? v * inv_s : v; };
        float v0 = w3(0) * (c - 1.5f * b * uu) + phys(d[0]);
        float sum = v0;
        d[0] = Elem<T>::kScaled ? v0 * s : v0;
#pragma unroll
        for (int i = 1; i < 19; i += 2) {
            const float eu = edot(ex3(i), ey3(i), ez3(i), u[0], u[1], u[2]);
            const float q = c + b * (4.5f * eu * eu - 1.5f * uu), t = a * eu;
            const float v1 = w3(i) * (q + t) + phys(d[i]);
            const float v2 = w3(i) * (q - t) + phys(d[i + 1]);
            sum += v1;
            sum += v2;
            d[i] = Elem<T>::kScaled ? v1 * s : v1;
            d[i + 1] = Elem<T>::kScaled ? v2 * s : v2;
        }
        inc = 0.0f;
        r = sum;
        return rb;
    }
    return rho;
}

template <typename T, int BCX, int BCY, int BCZ>
__device__ __forceinline__ float macro_node3(const char *src, const Layout &lay, const char *med,
                                             const MLayout &mlay, const Geom3 &g,
                                             const Physics3 &p3, float s, float inv_s, int y,
                                             int z, uint32_t x, float (&u)[3], float &r)
{
    const Rows3 R = rows3_of<BCY, BCZ>(src, lay, g, y, z);
    const Med3 md{make_rsrc(med + row3(g, y, z) * mlay.row, (uint32_t)mlay.row), mlay.slot,
                  2 * mlay.slot};
    float d[19], inc;
    const float rho = post_stream3<T, BCX>(R, lay, md, g, p3, s, inv_s, x, d, inc, r);
    float j[3], F[3];
    momentum3(d, j);
    if (Elem<T>::kScaled) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
            j[a] *= inv_s;
    }
    velocity3(p3, rho, j, md.eps(x), md.drag(x), md.kn0(x), u, F);
    return rho;
}

template <typename T, int BCX, int BCY, int BCZ>
__global__ __launch_bounds__(kBlock3) void sweep3_kernel(const char *src, char *dst, Layout lay,
                                                          const char *med, MLayout mlay,
                                                          Geom3 g, Physics3 p3, float s,
                                                          float inv_s, int bpr)
{
    const Node3 nd = node3_of(g, bpr);
    if (nd.x >= (uint32_t)g.nx)
        return;
    const Rows3 R = rows3_of<BCY, BCZ>(src, lay, g, nd.y, nd.z);
    const uint64_t row = row3(g, nd.y, nd.z);
    const Med3 md{make_rsrc(med + row * mlay.row, (uint32_t)mlay.row), mlay.slot,
                  2 * mlay.slot};
    float d[19], inc, r;
    const float rho = post_stream3<T, BCX>(R, lay, md, g, p3, s, inv_s, nd.x, d, inc, r);
    float j[3], u[3], F[3];
    momentum3(d, j);
    if (Elem<T>::kScaled) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
            j[a] *= inv_s;
    }
    const float eps = md.eps(nd.x);
    velocity3(p3, rho, j, eps, md.drag(nd.x), md.kn0(nd.x), u, F);
    float hs[19];
    collide3<T>(p3.ph, rho, inc, r, d, u, F, eps, s, hs);
    const Rsrc out = make_rsrc(dst + row * lay.row, (uint32_t)lay.row);
    st_f32(out, nd.x * 4, 0, rho, true);
    constexpr uint32_t es = sizeof(T);
#pragma unroll
    for (int i = 0; i < 19; ++i)
        Elem<T>::st(out, nd.x * es, lay.h_off + i * lay.h_slot, hs[i]);
}

// Read-out: rho, u into [nz][ny][nx] buffers (any may be NULL) and per-block
// FP64 partials [MAC_SLOTS][blocks] (MAC_DU2 unused).
template <typename T, int BCX, int BCY, int BCZ>
__global__ __launch_bounds__(kBlock3) void macro3_kernel(const char *src, Layout lay,
                                                          const char *med, MLayout mlay,
                                                          Geom3 g, Physics3 p3, float s,
                                                          float inv_s, int bpr, float *rho_out,
                                                          float *ux_out, float *uy_out,
                                                          float *uz_out, double *partials)
{
    __shared__ double sh[kBlock3 / 64];
    const Node3 nd = node3_of(g, bpr);
    double v[MAC_SLOTS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (nd.x < (uint32_t)g.nx) {
        float u[3], r;
        const float rho = macro_node3<T, BCX, BCY, BCZ>(src, lay, med, mlay, g, p3, s, inv_s,
                                                        nd.y, nd.z, nd.x, u, r);
        const double rp = (double)rho + (double)r;
        const uint64_t o = row3(g, nd.y, nd.z) * (uint64_t)g.nx + nd.x;
        if (rho_out)
            rho_out[o] = (float)rp;
        if (ux_out)
            ux_out[o] = u[0];
        if (uy_out)
            uy_out[o] = u[1];
        if (uz_out)
            uz_out[o] = u[2];
        v[MAC_FLUX] = rp * (double)u[0];
        v[MAC_UX] = u[0];
        v[MAC_U2] = (double)u[0] * u[0] + (double)u[1] * u[1] + (double)u[2] * u[2];
        v[MAC_RHO] = rp;
        v[MAC_QOUT] = (nd.x == (uint32_t)g.nx - 1) ? rp * (double)u[0] : 0.0;
    }
    const int L = xcd_remap3(blockIdx.x, gridDim.x);
#pragma unroll
    for (int k = 0; k < MAC_SLOTS; ++k) {
        const double rr = block_sum(v[k], sh);
        if (threadIdx.x == 0)
            partials[(int64_t)k * gridDim.x + L] = rr;
    }
}

// FP64 mass sum (rho + sum h / s), max |h| and the count of non-finite
// values, per block [ST_SLOTS][blocks].
template <typename T>
__global__ __launch_bounds__(kBlock3) void state_sums3_kernel(const char *src, Layout lay,
                                                               Geom3 g, float inv_s, int bpr,
                                                               double *partials)
{
    __shared__ double sh[kBlock3 / 64];
    const Node3 nd = node3_of(g, bpr);
    double mass = 0.0, hmax = 0.0, bad = 0.0;
    if (nd.x < (uint32_t)g.nx) {
        const Rsrc row = make_rsrc(src + row3(g, nd.y, nd.z) * lay.row, (uint32_t)lay.row);
        const float rho = ld_f32(row, nd.x * 4, 0);
        double hs = 0.0;
        bad += isfinite(rho) ? 0.0 : 1.0;
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const float h = Elem<T>::template ld<kAux3>(row, nd.x * sizeof(T), lay.h_off + i * lay.h_slot);
            bad += isfinite(h) ? 0.0 : 1.0;
            hs += (double)h;
            const double a = fabs((double)h * inv_s);
            hmax = a > hmax ? a : hmax;
        }
        mass = (double)rho + hs * inv_s;
    }
    const int L = xcd_remap3(blockIdx.x, gridDim.x);
    double r = block_sum(mass, sh);
    if (threadIdx.x == 0)
        partials[(int64_t)ST_MASS * gridDim.x + L] = r;
    r = block_max(hmax, sh);
    if (threadIdx.x == 0)
        partials[(int64_t)ST_HMAX * gridDim.x + L] = r;
    r = block_sum(bad, sh);
    if (threadIdx.x == 0)
        partials[(int64_t)ST_BAD * gridDim.x + L] = r;
}

// Rest (or the linear density ramp along x) with the FP64 density split
// into an FP32 value and its residual in the deviations.
template <typename T>
__global__ __launch_bounds__(kBlock3) void init3_kernel(char *dst, Layout lay, Geom3 g,
                                                         int ramp, double rho0, double rho_in,
                                                         double rho_out, float s, int bpr)
{
    const Node3 nd = node3_of(g, bpr);
    if (nd.x >= (uint32_t)g.nx)
        return;
    double rho = rho0;
    if (ramp)
        rho = g.nx > 1 ? rho_in + (rho_out - rho_in) * (double)nd.x / (double)(g.nx - 1)
                       : rho_in;
    const float hi = (float)rho;
    const float lo = (float)(rho - (double)hi);
    const Rsrc row = make_rsrc(dst + row3(g, nd.y, nd.z) * lay.row, (uint32_t)lay.row);
    st_f32(row, nd.x * 4, 0, hi, false);
#pragma unroll
    for (int i = 0; i < 19; ++i)
        Elem<T>::st(row, nd.x * sizeof(T), lay.h_off + i * lay.h_slot, w3(i) * lo * s);
}

// f*_i = w_i rho + h_i / s in FP64, [19][nz][ny][nx].
template <typename T>
__global__ __launch_bounds__(kBlock3) void populations3_kernel(const char *src, Layout lay,
                                                                Geom3 g, float inv_s, int bpr,
                                                                double *out)
{
    const Node3 nd = node3_of(g, bpr);
    if (nd.x >= (uint32_t)g.nx)
        return;
    const uint64_t rw = row3(g, nd.y, nd.z);
    const Rsrc row = make_rsrc(src + rw * lay.row, (uint32_t)lay.row);
    const double rho = ld_f32(row, nd.x * 4, 0);
    const uint64_t n = (uint64_t)g.nx * g.ny * g.nz, o = rw * g.nx + nd.x;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const float h = Elem<T>::template ld<kAux3>(row, nd.x * sizeof(T), lay.h_off + i * lay.h_slot);
        out[(uint64_t)i * n + o] = (double)w3(i) * rho + (double)h * inv_s;
    }
}

// Exact power-of-two rescale of the stored deviations (FP16 scale).
template <typename T>
__global__ __launch_bounds__(kBlock3) void rescale3_kernel(char *st, Layout lay, Geom3 g, int k,
                                                            int bpr)
{
    const Node3 nd = node3_of(g, bpr);
    if (nd.x >= (uint32_t)g.nx)
        return;
    const Rsrc row = make_rsrc(st + row3(g, nd.y, nd.z) * lay.row, (uint32_t)lay.row);
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const uint32_t off = lay.h_off + i * lay.h_slot;
        const float h = Elem<T>::template ld<kAux3>(row, nd.x * sizeof(T), off);
        Elem<T>::st(row, nd.x * sizeof(T), off, ldexpf(h, k));
    }
}

// Medium validation and k -> drag (0 where k = +inf or eps = 0), counting
// invalid values into partials [FLD_SLOTS][blocks].
__global__ __launch_bounds__(kBlock3) void fields3_kernel(char *med, MLayout mlay, Geom3 g,
                                                           double nu, double *partials, int bpr)
{
    __shared__ double sh[kBlock3 / 64];
    const Node3 nd = node3_of(g, bpr);
    double bad = 0.0;
    if (nd.x < (uint32_t)g.nx) {
        const Rsrc row = make_rsrc(med + row3(g, nd.y, nd.z) * mlay.row, (uint32_t)mlay.row);
        const float e = ld_f32(row, nd.x * 4, 0), k = ld_f32(row, nd.x * 4, mlay.slot),
                    kn = ld_f32(row, nd.x * 4, 2 * mlay.slot);
        const bool ok = (e >= 0.0f && e <= 1.0f) && (k > 0.0f) && (kn >= 0.0f && isfinite(kn));
        bad = ok ? 0.0 : 1.0;
        const float drag = (!ok || isinf(k) || e == 0.0f) ? 0.0f : (float)((double)e * nu / k);
        st_f32(row, nd.x * 4, mlay.slot, drag, false);
    }
    const int L = xcd_remap3(blockIdx.x, gridDim.x);
    const double r = block_sum(bad, sh);
    if (threadIdx.x == 0)
        partials[(int64_t)FLD_BAD * gridDim.x + L] = r;
}

} // namespace

int blocks3_of(const Geom3 &g) { return ((g.nx + kBlock3 - 1) / kBlock3) * g.ny * g.nz; }

#define LBK3_BC(FN, T, ...)                                                                  \
    switch (bcx * 4 + bcy * 2 + bcz) {                                                       \
    case 0: return FN<T, BC_PERIODIC, BC_PERIODIC, BC_PERIODIC>(__VA_ARGS__);                \
    case 1: return FN<T, BC_PERIODIC, BC_PERIODIC, BC_WALL>(__VA_ARGS__);                    \
    case 2: return FN<T, BC_PERIODIC, BC_WALL, BC_PERIODIC>(__VA_ARGS__);                    \
    case 3: return FN<T, BC_PERIODIC, BC_WALL, BC_WALL>(__VA_ARGS__);                        \
    case 4: return FN<T, BC_WALL, BC_PERIODIC, BC_PERIODIC>(__VA_ARGS__);                    \
    case 5: return FN<T, BC_WALL, BC_PERIODIC, BC_WALL>(__VA_ARGS__);                        \
    case 6: return FN<T, BC_WALL, BC_WALL, BC_PERIODIC>(__VA_ARGS__);                        \
    case 7: return FN<T, BC_WALL, BC_WALL, BC_WALL>(__VA_ARGS__);                            \
    case 8: return FN<T, BC_PRESSURE, BC_PERIODIC, BC_PERIODIC>(__VA_ARGS__);                \
    case 9: return FN<T, BC_PRESSURE, BC_PERIODIC, BC_WALL>(__VA_ARGS__);                    \
    case 10: return FN<T, BC_PRESSURE, BC_WALL, BC_PERIODIC>(__VA_ARGS__);                   \
    case 11: return FN<T, BC_PRESSURE, BC_WALL, BC_WALL>(__VA_ARGS__);                       \
    default: return hipErrorInvalidValue;                                                    \
    }

#define LBK3_DISPATCH(FN, ...)                                                               \
    if (bcx < 0 || bcx > 2 || bcy < 0 || bcy > 1 || bcz < 0 || bcz > 1)                      \
        return hipErrorInvalidValue;                                                         \
    switch (storage) {                                                                       \
    case 0: LBK3_BC(FN, float, __VA_ARGS__)                                                  \
    case 1: LBK3_BC(FN, __half, __VA_ARGS__)                                                 \
    case 2: LBK3_BC(FN, __hip_bfloat16, __VA_ARGS__)                                         \
    default: return hipErrorInvalidValue;                                                    \
    }

#define LBK3_T(KERNEL, ...)                                                                  \
    switch (storage) {                                                                       \
    case 0:                                                                                  \
        hipLaunchKernelGGL((KERNEL<float>), dim3(blocks3_of(g)), dim3(kBlock3), 0, st,       \
                           __VA_ARGS__, bpr);                                                \
        break;                                                                               \
    case 1:                                                                                  \
        hipLaunchKernelGGL((KERNEL<__half>), dim3(blocks3_of(g)), dim3(kBlock3), 0, st,      \
                           __VA_ARGS__, bpr);                                                \
        break;                                                                               \
    case 2:                                                                                  \
        hipLaunchKernelGGL((KERNEL<__hip_bfloat16>), dim3(blocks3_of(g)), dim3(kBlock3), 0,  \
                           st, __VA_ARGS__, bpr);                                            \
        break;                                                                               \
    default: return hipErrorInvalidValue;                                                    \
    }

template <typename T, int BCX, int BCY, int BCZ>
static hipError_t sweep3_t(const char *src, char *dst, const Layout &lay, const char *med,
                           const MLayout &mlay, const Geom3 &g, const Physics3 &p3, float s,
                           float inv_s, hipStream_t st)
{
    const int bpr = (g.nx + kBlock3 - 1) / kBlock3;
    hipLaunchKernelGGL((sweep3_kernel<T, BCX, BCY, BCZ>), dim3(blocks3_of(g)), dim3(kBlock3), 0,
                       st, src, dst, lay, med, mlay, g, p3, s, inv_s, bpr);
    return hipGetLastError();
}

template <typename T, int BCX, int BCY, int BCZ>
static hipError_t macro3_t(const char *src, const Layout &lay, const char *med,
                           const MLayout &mlay, const Geom3 &g, const Physics3 &p3, float s,
                           float inv_s, float *rho, float *ux, float *uy, float *uz,
                           double *partials, hipStream_t st)
{
    const int bpr = (g.nx + kBlock3 - 1) / kBlock3;
    hipLaunchKernelGGL((macro3_kernel<T, BCX, BCY, BCZ>), dim3(blocks3_of(g)), dim3(kBlock3), 0,
                       st, src, lay, med, mlay, g, p3, s, inv_s, bpr, rho, ux, uy, uz, partials);
    return hipGetLastError();
}

hipError_t launch_sweep3(int storage, int bcx, int bcy, int bcz, const char *src, char *dst,
                         const Layout &lay, const char *med, const MLayout &mlay,
                         const Geom3 &g, const Physics3 &p3, float s, float inv_s,
                         hipStream_t st)
{
    LBK3_DISPATCH(sweep3_t, src, dst, lay, med, mlay, g, p3, s, inv_s, st)
}

hipError_t launch_macro3(int storage, int bcx, int bcy, int bcz, const char *src,
                         const Layout &lay, const char *med, const MLayout &mlay,
                         const Geom3 &g, const Physics3 &p3, float s, float inv_s, float *rho,
                         float *ux, float *uy, float *uz, double *partials, hipStream_t st)
{
    LBK3_DISPATCH(macro3_t, src, lay, med, mlay, g, p3, s, inv_s, rho, ux, uy, uz, partials, st)
}

hipError_t launch_state_sums3(int storage, const char *src, const Layout &lay, const Geom3 &g,
                              float inv_s, double *partials, hipStream_t st)
{
    const int bpr = (g.nx + kBlock3 - 1) / kBlock3;
    switch (storage) {
    case 0:
        hipLaunchKernelGGL((state_sums3_kernel<float>), dim3(blocks3_of(g)), dim3(kBlock3), 0,
                           st, src, lay, g, inv_s, bpr, partials);
        break;
    case 1:
        hipLaunchKernelGGL((state_sums3_kernel<__half>), dim3(blocks3_of(g)), dim3(kBlock3), 0,
                           st, src, lay, g, inv_s, bpr, partials);
        break;
    case 2:
        hipLaunchKernelGGL((state_sums3_kernel<__hip_bfloat16>), dim3(blocks3_of(g)),
                           dim3(kBlock3), 0, st, src, lay, g, inv_s, bpr, partials);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_init3(int storage, char *dst, const Layout &lay, const Geom3 &g, int ramp,
                        double rho0, double rho_in, double rho_out, float s, hipStream_t st)
{
    const int bpr = (g.nx + kBlock3 - 1) / kBlock3;
    LBK3_T(init3_kernel, dst, lay, g, ramp, rho0, rho_in, rho_out, s)
    return hipGetLastError();
}

hipError_t launch_populations3(int storage, const char *src, const Layout &lay, const Geom3 &g,
                               float inv_s, double *out, hipStream_t st)
{
    const int bpr = (g.nx + kBlock3 - 1) / kBlock3;
    switch (storage) {
    case 0:
        hipLaunchKernelGGL((populations3_kernel<float>), dim3(blocks3_of(g)), dim3(kBlock3), 0,
                           st, src, lay, g, inv_s, bpr, out);
        break;
    case 1:
        hipLaunchKernelGGL((populations3_kernel<__half>), dim3(blocks3_of(g)), dim3(kBlock3), 0,
                           st, src, lay, g, inv_s, bpr, out);
        break;
    case 2:
        hipLaunchKernelGGL((populations3_kernel<__hip_bfloat16>), dim3(blocks3_of(g)),
                           dim3(kBlock3), 0, st, src, lay, g, inv_s, bpr, out);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_rescale3(int storage, char *state, const Layout &lay, const Geom3 &g, int k,
                           hipStream_t st)
{
    const int bpr = (g.nx + kBlock3 - 1) / kBlock3;
    LBK3_T(rescale3_kernel, state, lay, g, k)
    return hipGetLastError();
}

hipError_t launch_fields3(char *med, const MLayout &mlay, const Geom3 &g, double nu,
                          double *partials, hipStream_t st)
{
    const int bpr = (g.nx + kBlock3 - 1) / kBlock3;
    hipLaunchKernelGGL(fields3_kernel, dim3(blocks3_of(g)), dim3(kBlock3), 0, st, med, mlay, g,
                       nu, partials, bpr);
    return hipGetLastError();
}

} // namespace lbk
