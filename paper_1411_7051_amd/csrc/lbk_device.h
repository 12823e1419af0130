// lbk_device.h -- device-side building blocks of the fused D2Q9 Klinkenberg
// sweep for gfx950: lattice constants, buffer-resource element I/O, the pull
// stream, the node velocity solve and the BGK/Guo collide, all written in
// the density-split form used by every storage type:
//
//   stored per node x:  rho(x) (FP32)   and   h_i(x) = f*_i(x) - w_i rho(x)
//
// so that the nine population slots carry only deviations from the local
// density.  The deviations are the small quantities the flow lives in (at
// the low Mach numbers of tight media they are 1e-12 .. 1e-4), and keeping
// them apart from the O(1) density gives every storage type its full
// relative precision on them.  Post-stream populations are handled as
// f_i = w_i rho_c + d_i with rho_c the node's stored density; the density
// update rho_c + sum d_i is split into its FP32-rounded value and the exact
// rounding residual (Fast2Sum), which stays in the deviations, so no mass is
// lost to rounding of the density.
//
// FP16 stores the deviations times a power of two s (the "scaled" unit);
// the arithmetic on deviations runs in that unit, with s folded into the
// per-direction-class constants, so the scale costs no per-population work.
//
// Memory access: every kernel maps one block to 256 consecutive x of one
// row, so each row's base is uniform.  Rows are reached through buffer
// resources (scalar registers) with a 32-bit per-lane byte offset: no
// per-access address arithmetic, and hardware range checking on every
// access (an out-of-range load returns 0 instead of faulting).
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbk {

enum { BC_PERIODIC = 0, BC_WALL = 1, BC_PRESSURE = 2 };

// D2Q9 velocities (Eq. 13): i = 0 rest, 1..4 axes at (i-1)pi/2,
// 5..8 diagonals at (i-5)pi/2 + pi/4.
__host__ __device__ constexpr int ex_of(int i)
{
    return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__host__ __device__ constexpr int ey_of(int i)
{
    return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}
__host__ __device__ constexpr int opp_of(int i)
{
    return i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5);
}
// e . a for a lattice velocity e (components -1, 0, 1): the terms of zero
// components are left out rather than multiplied by 0 (a product the
// compiler must keep, since 0 * inf is NaN); the others are summed in order.
__device__ __forceinline__ float edot(int ex, int ey, int ez, float ax, float ay, float az)
{
    float v = 0.0f;
    bool first = true;
    if (ex != 0) {
        v = ex * ax;
        first = false;
    }
    if (ey != 0) {
        v = first ? ey * ay : v + ey * ay;
        first = false;
    }
    if (ez != 0)
        v = first ? ez * az : v + ez * az;
    return v;
}

// Weights stated with Eq. 14.
__host__ __device__ constexpr float w_of(int i)
{
    return i == 0 ? 4.0f / 9.0f : (i <= 4 ? 1.0f / 9.0f : 1.0f / 36.0f);
}

static_assert(opp_of(1) == 3 && opp_of(2) == 4 && opp_of(5) == 7 && opp_of(6) == 8 &&
                  opp_of(7) == 5 && opp_of(8) == 6 && opp_of(3) == 1 && opp_of(4) == 2,
              "opposite directions");

// ---------------------------------------------------------- buffer I/O

typedef __amdgpu_buffer_rsrc_t Rsrc;
// Raw (unstructured) buffer descriptor word 3 for the gfx9 family.
constexpr int kRsrcWord3 = 0x00020000;
// Cache policy of the population streams: nontemporal.  Each stored
// population is read once and written once per step; the density and the
// medium, whose neighbour reads reuse, keep the default policy.  Population
// loads take the policy as a template argument (a sweep whose density
// reuse spans more rows than stay cached passes the default policy).
constexpr int kNT = 2;

__device__ __forceinline__ Rsrc make_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             kRsrcWord3);
}
__device__ __forceinline__ float ld_f32(Rsrc r, uint32_t voff, uint32_t soff)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ float ld_f32_nt(Rsrc r, uint32_t voff, uint32_t soff)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, kNT));
}
__device__ __forceinline__ void st_f32(Rsrc r, uint32_t voff, uint32_t soff, float v, bool nt)
{
    if (nt)
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)voff, (int)soff, kNT);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)voff, (int)soff, 0);
}

// The adjoint's history of one node: (rho, jx, jy) as three consecutive FP32
// values, moved with one 96-bit access.
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
template <int AUX>
__device__ __forceinline__ void ld_hist(Rsrc r, uint32_t voff, float (&h)[3])
{
    const u32x3 v = __builtin_amdgcn_raw_buffer_load_b96(r, (int)voff, 0, AUX);
    h[0] = __uint_as_float(v.x);
    h[1] = __uint_as_float(v.y);
    h[2] = __uint_as_float(v.z);
}
template <int AUX>
__device__ __forceinline__ void st_hist(Rsrc r, uint32_t voff, float rho, float jx, float jy)
{
    u32x3 v;
    v.x = __float_as_uint(rho);
    v.y = __float_as_uint(jx);
    v.z = __float_as_uint(jy);
    __builtin_amdgcn_raw_buffer_store_b96(v, r, (int)voff, 0, AUX);
}

// v as an opaque FP32 register value.  The compiler may otherwise fold the
// rounding of an FP32 result to FP16 into the arithmetic that produced it
// (a mixed-precision FMA that rounds once, straight to FP16), and may do so
// in one kernel and not in another; every FP16 store and its register
// stand-in round through this, so all kernels round first to FP32 and then
// to FP16, identically.
__device__ __forceinline__ float f32_reg(float v)
{
    asm("" : "+v"(v));
    return v;
}

// Storage element types, loaded and stored in the storage's own unit
// (scaled for FP16).
template <typename T> struct Elem;
template <> struct Elem<float> {
    static constexpr bool kScaled = false;
    template <int AUX = kNT>
    static __device__ __forceinline__ float ld(Rsrc r, uint32_t voff, uint32_t soff)
    {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, AUX));
    }
    template <int AUX = kNT>
    static __device__ __forceinline__ void st(Rsrc r, uint32_t voff, uint32_t soff, float v)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)voff, (int)soff, AUX);
    }
    // the value a store followed by a load returns
    static __device__ __forceinline__ float round(float v) { return v; }
};
template <> struct Elem<__half> {
    static constexpr bool kScaled = true;
    template <int AUX = kNT>
    static __device__ __forceinline__ float ld(Rsrc r, uint32_t voff, uint32_t soff)
    {
        const uint16_t u = __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, AUX);
        return __half2float(__ushort_as_half(u));
    }
    template <int AUX = kNT>
    static __device__ __forceinline__ void st(Rsrc r, uint32_t voff, uint32_t soff, float v)
    {
        __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(__float2half_rn(f32_reg(v))), r,
                                              (int)voff, (int)soff, AUX);
    }
    static __device__ __forceinline__ float round(float v)
    {
        return __half2float(__float2half_rn(f32_reg(v)));
    }
};
template <> struct Elem<__hip_bfloat16> {
    static constexpr bool kScaled = false;
    template <int AUX = kNT>
    static __device__ __forceinline__ float ld(Rsrc r, uint32_t voff, uint32_t soff)
    {
        const uint16_t u = __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, AUX);
        return __uint_as_float((uint32_t)u << 16);
    }
    template <int AUX = kNT>
    static __device__ __forceinline__ void st(Rsrc r, uint32_t voff, uint32_t soff, float v)
    {
        const __hip_bfloat16 b = __float2bfloat16(v); // round to nearest even
        __builtin_amdgcn_raw_buffer_store_b16(*reinterpret_cast<const uint16_t *>(&b), r,
                                              (int)voff, (int)soff, AUX);
    }
    static __device__ __forceinline__ float round(float v)
    {
        const __hip_bfloat16 b = __float2bfloat16(v);
        return __uint_as_float((uint32_t)(*reinterpret_cast<const uint16_t *>(&b)) << 16);
    }
};

// Value of v held by the lane DX to the left (DX = 1: lane - 1) or right
// (DX = -1: lane + 1) within the wave64, through a whole-wave DPP shift
// (wave_shr:1 / wave_shl:1); DX = 0 is v itself.  The lane at the wave's
// edge, which has no such neighbour, gets 0 through the shift's bound
// control (rather than from a destination cleared beforehand, which cost
// one more instruction per shift).
template <int DX> __device__ __forceinline__ float lane_from(float v)
{
    if (DX == 1)
        return __int_as_float(
            __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
    if (DX == -1)
        return __int_as_float(
            __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
    return v;
}

// -------------------------------------------------------------- layouts

// Scalars of one run, precomputed on the host in FP64 and rounded once.
struct Physics {
    float omega;     // 1/tau
    float guo;       // 1 - 1/(2 tau), the factor of Eq. 15
    float gx, gy;    // G of Eq. 8
    float feps;      // Forchheimer function of Eq. 2 (0: Eq. 8)
    float inv_nu;    // 1/nu (Forchheimer term only)
    float rho_ref;   // density at which kn0 is quoted
    float rin_hi, rin_lo;   // rho_in = hi + lo exactly (FP64 -> 2 x FP32)
    float rout_hi, rout_lo; // rho_out likewise
    int kn_local;
    int corr;        // slip correlation: CORR_BKC, CORR_KLINKENBERG, CORR_NONE
    float slip_nb;   // -b, b the slip coefficient of Eq. 6
    float slip_c;    // 4 - b
};

enum { CORR_BKC = 0, CORR_KLINKENBERG = 1, CORR_NONE = 2 };

// Correction factor of the selected correlation as a ratio f_c = den / num
// (one reciprocal serves f_c and the velocity solve):
//   CORR_BKC (Eqs. 6-7): with t = Kn^0.4348 and a = t + 0.170,
//     1 + alpha Kn = (a + 1.358 t Kn) / a and
//     1 + 4 Kn / (1 - b Kn) = (1 + (4 - b) Kn) / (1 - b Kn);
//   CORR_KLINKENBERG (Eqs. 4-5): 1 + 4 Kn;  CORR_NONE: 1.
// t = exp2(0.4348 log2 Kn) is 0 at Kn = 0, so f_c(0) = 1.
__device__ __forceinline__ float fc_pow(float kn)
{
    return __builtin_amdgcn_exp2f(0.4348f * __builtin_amdgcn_logf(kn));
}
// fc_parts with t = fc_pow(kn) given (used only by CORR_BKC).
__device__ __forceinline__ void fc_parts_t(const Physics &ph, float kn, float t, float &num,
                                           float &den)
{
    if (ph.corr == CORR_BKC) {
        const float a = t + 0.170f;
        num = a * (1.0f + ph.slip_nb * kn);
        den = (a + 1.358f * t * kn) * (1.0f + ph.slip_c * kn);
    } else if (ph.corr == CORR_KLINKENBERG) {
        num = 1.0f;
        den = 1.0f + 4.0f * kn;
    } else {
        num = 1.0f;
        den = 1.0f;
    }
}
__device__ __forceinline__ void fc_parts(const Physics &ph, float kn, float &num, float &den)
{
    if (ph.corr == CORR_BKC)
        fc_parts_t(ph, kn, fc_pow(kn), num, den);
    else
        fc_parts_t(ph, kn, 0.0f, num, den);
}

// Lattice extent; `pitch` = elements per row slot (a multiple of 64).
struct Geom {
    int nx, ny, pitch;
};

// Byte layout of one time level of the state: row block y starts at
// y * row and holds the density (FP32) at offset 0 and h_i (T) at
// h_off + i * h_slot.
struct Layout {
    uint64_t row;
    uint32_t h_off;
    uint32_t h_slot;
};

// Byte layout of the read-only medium: row block y starts at y * row and
// holds eps at 0, drag = eps nu / k (0 where k = +inf) at slot, kn0 at
// 2 slot (FP32).
struct MLayout {
    uint64_t row;
    uint32_t slot;
};

template <typename T> __device__ __forceinline__ Rsrc state_row(const char *base, const Layout &L,
                                                                int y)
{
    return make_rsrc(base + (uint64_t)y * L.row, (uint32_t)L.row);
}
__device__ __forceinline__ Rsrc med_row(const char *base, const MLayout &M, int y)
{
    return make_rsrc(base + (uint64_t)y * M.row, (uint32_t)M.row);
}

// The three rows a node pulls from, and whether the row below / above lies
// beyond a wall (then the node's own row stands in; its entries are unused).
struct Rows {
    Rsrc r[3];
    bool wym, wyp;
};

template <int BCY>
__device__ __forceinline__ Rows rows_of(const char *base, const Layout &L, const Geom &g, int y)
{
    int ym = y - 1, yp = y + 1;
    Rows R;
    if (BCY == BC_PERIODIC) {
        ym = (y == 0) ? g.ny - 1 : ym;
        yp = (y == g.ny - 1) ? 0 : yp;
        R.wym = R.wyp = false;
    } else {
        // the row is the same for the whole workgroup: read the wall flags
        // through a scalar register, so that selects on them stay scalar
        // (a lane-mask select of a buffer resource becomes a waterfall loop)
        R.wym = __builtin_amdgcn_readfirstlane(y == 0 ? 1 : 0) != 0;
        R.wyp = __builtin_amdgcn_readfirstlane(y == g.ny - 1 ? 1 : 0) != 0;
        ym = R.wym ? y : ym;
        yp = R.wyp ? y : yp;
    }
    R.r[0] = make_rsrc(base + (uint64_t)ym * L.row, (uint32_t)L.row);
    R.r[1] = make_rsrc(base + (uint64_t)y * L.row, (uint32_t)L.row);
    R.r[2] = make_rsrc(base + (uint64_t)yp * L.row, (uint32_t)L.row);
    return R;
}

// Pull-stream of node (x, y): post-stream deviations d_i = f_i - w_i rc in
// the storage unit (times s for FP16), with rc the node's stored density.
// A link that crosses a wall returns the node's own opposite deviation
// (half-way bounce-back); periodic axes wrap.  Pressure columns are never
// pulled for themselves (the caller pulls their neighbour instead), so
// x - 1 and x + 1 stay inside the row there.
template <typename T, int BCX>
__device__ __forceinline__ void pull(const Rows &R, const Layout &L, const Geom &g, float s,
                                     uint32_t x, float &rc, float (&d)[9])
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
    rc = ld_f32(R.r[1], x * 4, 0);
    d[0] = Elem<T>::ld(R.r[1], x * es, L.h_off);
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const int ex = ex_of(i), ey = ey_of(i);
        const uint32_t sx = ex == 1 ? xm : (ex == -1 ? xp : x);
        const bool wall_y = (ey == 1 && R.wym) || (ey == -1 && R.wyp); // uniform
        const float ws = Elem<T>::kScaled ? w_of(i) * s : w_of(i);
        // a wall link reads the node's own opposite slot; its density term
        // is then rho(x) - rc = 0 exactly, so one expression serves both
        // (uniform selects of the row and slot, no divergent load)
        const int ry = ey == 1 ? 0 : (ey == -1 ? 2 : 1);
        const Rsrc src = wall_y ? R.r[1] : R.r[ry];
        const uint32_t vx = wall_y ? x : sx;
        const uint32_t so = L.h_off + (uint32_t)(wall_y ? opp_of(i) : i) * L.h_slot;
        const float rn = ld_f32(src, vx * 4, 0);
        const float h = Elem<T>::ld(src, vx * es, so);
        d[i] = ws * (rn - rc) + h;
        if (BCX == BC_WALL) {
            const bool wall_x = (ex == 1 && wxm) || (ex == -1 && wxp); // per lane, edges only
            if (wall_x)
                d[i] = Elem<T>::ld(R.r[1], x * es, L.h_off + opp_of(i) * L.h_slot);
        }
    }
}

// Density update of a pulled node: s_phys = sum d / s; rho = FP32(rc +
// s_phys); inc = rho - rc (exact, Sterbenz); r = s_phys - inc, the exact
// rounding residual (Fast2Sum with |rc| >= |s_phys|).  The deviations
// relative to rho are d_i - w_i inc; they are never formed explicitly.
template <typename T>
__device__ __forceinline__ float density(float rc, const float (&d)[9], float inv_s, float &inc,
                                         float &r)
{
    float sum = 0.0f;
#pragma unroll
    for (int i = 0; i < 9; ++i)
        sum += d[i];
    const float sp = Elem<T>::kScaled ? sum * inv_s : sum;
    const float rho = rc + sp;
    inc = rho - rc;
    r = sp - inc;
    return rho;
}

// sum_i e_i d_i, in the storage unit (the weights' part cancels in pairs).
__device__ __forceinline__ void momentum(const float (&d)[9], float &jx, float &jy)
{
    jx = (d[1] - d[3]) + (d[5] - d[7]) + (d[8] - d[6]);
    jy = (d[2] - d[4]) + (d[5] - d[7]) + (d[6] - d[8]);
}

// Velocity and force of one node from rho and j = sum f e: Eq. 16b solved
// as Eq. 17 (or the Forchheimer quadratic of Eq. 2), with the apparent
// permeability k_a = k f_c(Kn) of Eq. 3 and Kn = kn0 rho_ref / rho.
//
// With t = Kn^0.4348 and a = t + 0.170, Eqs. 6-7 (b = -1) read
//   f_c = (a + 1.358 t Kn)(1 + 5 Kn) / (a (1 + Kn)) = den / num,
// finite and equal to 1 at Kn = 0 (t = 0).  The Darcy coefficient is
// A = drag / f_c = drag num / den, and Eq. 17 gives u = v / (1 + A/2) with
// v = j / rho + eps G / 2, so one reciprocal R = 1 / (2 den + drag num)
// yields both u = 2 den R v and A u = 2 drag num R v.
// eps = 0: u = 0 and rho F = -2 j (the infinite-drag limit of Eq. 17).
__device__ __forceinline__ void velocity(const Physics &ph, float rho, float jx, float jy,
                                         float eps, float drag, float kn0, float &ux, float &uy,
                                         float &Fx, float &Fy)
{
    const float rinv = __builtin_amdgcn_rcpf(rho);
    const float kn = ph.kn_local ? kn0 * (ph.rho_ref * rinv) : kn0;
    float num, den;
    fc_parts(ph, kn, num, den);
    const float egx = eps * ph.gx, egy = eps * ph.gy;
    const float vx = jx * rinv + 0.5f * egx;
    const float vy = jy * rinv + 0.5f * egy;
    float g, ag, B = 0.0f;
    if (ph.feps == 0.0f) {
        const float dn = drag * num;
        const float R2 = 2.0f * __builtin_amdgcn_rcpf(2.0f * den + dn);
        g = den * R2;
        ag = dn * R2;
    } else {
        // Forchheimer (Eq. 2): (1 + A/2) u + (B/2) |u| u = v with
        // B = eps F_eps / sqrt(k_a), k_a = eps nu / A; positive root of
        // the quadratic in |u|, rationalized.
        const float A = drag * num * __builtin_amdgcn_rcpf(den);
        B = ph.feps * __builtin_sqrtf(eps * A * ph.inv_nu);
        const float c0 = 1.0f + 0.5f * A;
        const float wn = __builtin_sqrtf(vx * vx + vy * vy);
        g = 2.0f / (c0 + __builtin_sqrtf(c0 * c0 + 2.0f * B * wn));
        ag = A * g;
    }
    const bool solid = !(eps > 0.0f);
    ux = solid ? 0.0f : g * vx;
    uy = solid ? 0.0f : g * vy;
    float fx = egx - ag * vx, fy = egy - ag * vy;
    if (ph.feps != 0.0f) {
        const float bu = B * __builtin_sqrtf(ux * ux + uy * uy);
        fx -= bu * ux;
        fy -= bu * uy;
    }
    Fx = solid ? -2.0f * jx * rinv : fx;
    Fy = solid ? -2.0f * jy * rinv : fy;
}

// BGK relaxation with Guo forcing (Eqs. 12, 14, 15) in deviation form.
// With delta_i = d_i - w_i inc the post-stream deviations from w_i rho,
//   h*_i = (1 - omega) delta_i + omega (w_i r + geq_i) + F_i,
// r the density residual, geq_i the Eq. 14 deviation and F_i Eq. 15.
// Over the pairs (i, opp i), with eu = e_i.u, eF = e_i.F, g = 1 - 1/(2 tau),
// P = omega eu + g eF and E = eu (P + g eF):
//   h*_i, h*_opp = (1 - omega) d_i + w_i C + w_i rho (4.5 E / eps +/- 3 P)
//   C = omega r - (1 - omega) inc + rho/eps (-1.5 omega u.u - 3 g u.F).
// d_i and the outputs are in the storage unit (times s for FP16).
// For eps = 0 the 1/eps terms vanish with u = 0.
template <typename T>
__device__ __forceinline__ void collide(const Physics &ph, float rho, float inc, float r,
                                        const float (&d)[9], float ux, float uy, float Fx,
                                        float Fy, float eps, float s, float (&hs)[9])
{
    const bool solid = !(eps > 0.0f);
    const float ie = solid ? 0.0f : __builtin_amdgcn_rcpf(eps);
    const float om = ph.omega, cg = ph.guo, keep = 1.0f - om;
    float C = om * r - keep * inc +
              rho * ie * (-1.5f * om * (ux * ux + uy * uy) - 3.0f * cg * (ux * Fx + uy * Fy));
    float rs = rho;
    if (Elem<T>::kScaled) {
        C *= s;
        rs *= s;
    }
    const float Kb = 4.5f * rs * ie, Mb = 3.0f * rs; // times w_i below
    hs[0] = keep * d[0] + w_of(0) * C;
#pragma unroll
    for (int i = 1; i <= 6; ++i) {
        if (i == 3 || i == 4)
            continue; // pairs (1,3) (2,4) (5,7) (6,8)
        const float w = w_of(i);
        const float eu = edot(ex_of(i), ey_of(i), 0, ux, uy, 0.0f);
        const float q = cg * edot(ex_of(i), ey_of(i), 0, Fx, Fy, 0.0f);
        const float P = om * eu + q;
        const float E = eu * (P + q);
        const float X = (w * Kb) * E + w * C;
        const float Y = (w * Mb) * P;
        hs[i] = keep * d[i] + (X + Y);
        hs[opp_of(i)] = keep * d[opp_of(i)] + (X - Y);
    }
}

} // namespace lbk
