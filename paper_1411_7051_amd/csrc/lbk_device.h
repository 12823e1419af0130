// lbk_device.h -- device-side building blocks of the fused D2Q9 Klinkenberg
// sweep for gfx950: lattice constants, storage element types, the pull
// stream, the node velocity solve and the BGK/Guo collide, all written in
// the density-split form used by every storage type:
//
//   stored per node x:  rho(x) (FP32)   and   h_i(x) = f*_i(x) - w_i rho(x)
//
// so that the nine planes carry only deviations from the local density.
// The deviations are the small quantities the flow lives in (at the low
// Mach numbers of tight media they are 1e-12 .. 1e-4), and keeping them
// apart from the O(1) density gives every storage type its full relative
// precision on them.  Post-stream populations are handled as
// f_i = w_i rho_c + d_i with rho_c the node's stored density, and the
// density update rho_new = rho_c + sum d_i is split into its FP32-rounded
// value and an exact residual that stays in the deviations, so no mass is
// lost to rounding of the density plane.
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
// Weights stated with Eq. 14.
__host__ __device__ constexpr float w_of(int i)
{
    return i == 0 ? 4.0f / 9.0f : (i <= 4 ? 1.0f / 9.0f : 1.0f / 36.0f);
}

static_assert(opp_of(1) == 3 && opp_of(2) == 4 && opp_of(5) == 7 && opp_of(6) == 8 &&
                  opp_of(7) == 5 && opp_of(8) == 6 && opp_of(3) == 1 && opp_of(4) == 2,
              "opposite directions");

// Storage element types.  FP16 values are the deviations times a power of
// two (scale), so that they sit in the normal FP16 range; BF16 and FP32
// need no scale.  Every stored population is read once and written once per
// step, so loads and stores are nontemporal: they bypass the caches' reuse
// policy and leave L2 to the density plane, whose neighbour reads do reuse.
template <typename T> struct Elem;
template <> struct Elem<float> {
    static __device__ __forceinline__ float ld(const float *p, int64_t i, float)
    {
        return __builtin_nontemporal_load(p + i);
    }
    static __device__ __forceinline__ void st(float *p, int64_t i, float v, float)
    {
        __builtin_nontemporal_store(v, p + i);
    }
};
template <> struct Elem<__half> {
    static __device__ __forceinline__ float ld(const __half *p, int64_t i, float inv_s)
    {
        const uint16_t u = __builtin_nontemporal_load(reinterpret_cast<const uint16_t *>(p) + i);
        return __half2float(__ushort_as_half(u)) * inv_s;
    }
    static __device__ __forceinline__ void st(__half *p, int64_t i, float v, float s)
    {
        __builtin_nontemporal_store(__half_as_ushort(__float2half_rn(v * s)),
                                    reinterpret_cast<uint16_t *>(p) + i);
    }
};
template <> struct Elem<__hip_bfloat16> {
    static __device__ __forceinline__ float ld(const __hip_bfloat16 *p, int64_t i, float)
    {
        const uint16_t u = __builtin_nontemporal_load(reinterpret_cast<const uint16_t *>(p) + i);
        return __uint_as_float((uint32_t)u << 16);
    }
    static __device__ __forceinline__ void st(__hip_bfloat16 *p, int64_t i, float v, float)
    {
        const __hip_bfloat16 b = __float2bfloat16(v); // round to nearest even
        __builtin_nontemporal_store(*reinterpret_cast<const uint16_t *>(&b),
                                    reinterpret_cast<uint16_t *>(p) + i);
    }
};

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
};

// Plane geometry: nx x ny nodes, rows of `pitch` elements, `plane` = ny*pitch.
struct Geom {
    int nx, ny, pitch;
    int64_t plane;
};

// Lattice state buffers of one time level.
template <typename T> struct State {
    float *rho; // [ny][pitch]
    T *h;       // [9][ny][pitch]
};

// Per-node medium: eps, drag = eps nu / k (0 where k = +inf), kn0.
struct Medium {
    const float *eps;
    const float *drag;
    const float *kn0;
};

// Beskok-Karniadakis/Civan factor (Eqs. 6-7, b = -1) in FP32 with the
// hardware log2/exp2; f_c = 1 at Kn = 0.
__device__ __forceinline__ float fc_of(float kn)
{
    // Kn^-0.4348 = exp2(-0.4348 log2 Kn)
    float p = __builtin_amdgcn_exp2f(-0.4348f * __builtin_amdgcn_logf(kn));
    float alpha = 1.358f * __builtin_amdgcn_rcpf(1.0f + 0.170f * p);
    float fc = (1.0f + alpha * kn) * (1.0f + 4.0f * kn * __builtin_amdgcn_rcpf(1.0f + kn));
    return kn > 0.0f ? fc : 1.0f;
}

// Pull-stream of node (x, y): post-stream deviations d_i = f_i - w_i rc,
// with rc the node's stored density.  A link that crosses a wall returns
// the node's own opposite deviation (half-way bounce-back); periodic axes
// wrap.  Pressure columns are never pulled for themselves (the caller pulls
// their neighbour instead), so x - 1 and x + 1 stay inside the row there.
template <typename T, int BCX, int BCY>
__device__ __forceinline__ void pull(const State<T> &src, const Geom &g, float inv_s, int x,
                                     int y, float &rc, float (&d)[9])
{
    int xm = x - 1, xp = x + 1, ym = y - 1, yp = y + 1;
    bool wxm = false, wxp = false, wym = false, wyp = false;
    if (BCX == BC_PERIODIC) {
        xm = (x == 0) ? g.nx - 1 : xm;
        xp = (x == g.nx - 1) ? 0 : xp;
    } else if (BCX == BC_WALL) {
        wxm = (x == 0);
        wxp = (x == g.nx - 1);
    }
    if (BCY == BC_PERIODIC) {
        ym = (y == 0) ? g.ny - 1 : ym;
        yp = (y == g.ny - 1) ? 0 : yp;
    } else {
        wym = (y == 0);
        wyp = (y == g.ny - 1);
    }
    const int c = y * g.pitch + x;
    rc = src.rho[c];
    d[0] = Elem<T>::ld(src.h, c, inv_s);
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const int ex = ex_of(i), ey = ey_of(i);
        const int sx = ex == 1 ? xm : (ex == -1 ? xp : x);
        const int sy = ey == 1 ? ym : (ey == -1 ? yp : y);
        const bool wall = (ex == 1 && wxm) || (ex == -1 && wxp) || (ey == 1 && wym) ||
                          (ey == -1 && wyp);
        // bounce-back reads the node's own opposite population; the density
        // difference is then zero
        const int n = wall ? c : sy * g.pitch + sx;
        const int plane = wall ? opp_of(i) : i;
        const float rn = src.rho[n];
        d[i] = w_of(i) * (rn - rc) + Elem<T>::ld(src.h + plane * g.plane, n, inv_s);
    }
}

// Split rho_c + sum d into its FP32 value and deviations relative to it:
// delta_i = d_i - w_i (rho - rc) with rho - rc exact (Sterbenz), so that
// w_i rho + delta_i = w_i rc + d_i holds to the rounding of the deviations.
__device__ __forceinline__ float split_density(float rc, const float (&d)[9], float (&dl)[9])
{
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < 9; ++i)
        s += d[i];
    const float rho = rc + s;
    const float inc = rho - rc;
#pragma unroll
    for (int i = 0; i < 9; ++i)
        dl[i] = d[i] - w_of(i) * inc;
    return rho;
}

__device__ __forceinline__ void momentum(const float (&dl)[9], float &jx, float &jy)
{
    jx = (dl[1] - dl[3]) + (dl[5] - dl[7]) + (dl[8] - dl[6]);
    jy = (dl[2] - dl[4]) + (dl[5] - dl[7]) + (dl[6] - dl[8]);
}

// Velocity and force of one node from rho and j = sum f e (Eq. 16b solved as
// Eq. 17, or the Forchheimer quadratic of Eq. 2), with k_a = k f_c(Kn) and
// Kn = kn0 rho_ref / rho.  eps = 0: u = 0 and rho F = -2 j (the infinite
// drag limit of Eq. 17).
__device__ __forceinline__ void velocity(const Physics &ph, float rho, float jx, float jy,
                                         float eps, float drag, float kn0, float &ux, float &uy,
                                         float &Fx, float &Fy)
{
    const float rinv = __builtin_amdgcn_rcpf(rho);
    const float kn = ph.kn_local ? kn0 * ph.rho_ref * rinv : kn0;
    const float fc = fc_of(kn);
    const float A = drag * __builtin_amdgcn_rcpf(fc); // eps nu / k_a
    const float vx = jx * rinv + 0.5f * eps * ph.gx;
    const float vy = jy * rinv + 0.5f * eps * ph.gy;
    const float c0 = 1.0f + 0.5f * A;
    float g, B = 0.0f;
    if (ph.feps != 0.0f) {
        // B = eps F_eps / sqrt(k_a), k_a = eps nu f_c / drag
        B = eps * ph.feps * __builtin_sqrtf(drag * ph.inv_nu * __builtin_amdgcn_rcpf(eps * fc));
        B = drag > 0.0f ? B : 0.0f;
        const float wn = __builtin_sqrtf(vx * vx + vy * vy);
        g = 2.0f / (c0 + __builtin_sqrtf(c0 * c0 + 2.0f * B * wn));
    } else {
        g = __builtin_amdgcn_rcpf(c0);
    }
    const bool solid = !(eps > 0.0f);
    ux = solid ? 0.0f : g * vx;
    uy = solid ? 0.0f : g * vy;
    const float un = __builtin_sqrtf(ux * ux + uy * uy);
    Fx = solid ? -2.0f * jx * rinv : -A * ux - B * un * ux + eps * ph.gx;
    Fy = solid ? -2.0f * jy * rinv : -A * uy - B * un * uy + eps * ph.gy;
}

// Equilibrium deviation of Eq. 14 from w_i rho:
// w_i rho [3 e.u + 9/(2 eps) (e.u)^2 - 3/(2 eps) u.u]; zero at eps = 0.
__device__ __forceinline__ void geq_dev(float rho, float ux, float uy, float eps,
                                        float (&ge)[9])
{
    const bool solid = !(eps > 0.0f);
    const float ie = solid ? 0.0f : __builtin_amdgcn_rcpf(eps);
    ux = solid ? 0.0f : ux;
    uy = solid ? 0.0f : uy;
    const float base = -1.5f * ie * (ux * ux + uy * uy);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const float eu = ex_of(i) * ux + ey_of(i) * uy;
        ge[i] = w_of(i) * rho * (3.0f * eu + 4.5f * ie * eu * eu + base);
    }
}

// BGK relaxation with Guo forcing (Eqs. 12, 14, 15) in deviation form:
//   h*_i = (1 - omega) dl_i + omega (w_i r + geq_i) + F_i
// where r = sum dl (the exact density residual) and geq_i is the Eq. 14
// deviation.  For eps = 0 the 1/eps terms vanish with u = 0.
__device__ __forceinline__ void collide(const Physics &ph, float rho, const float (&dl)[9],
                                        float ux, float uy, float Fx, float Fy, float eps,
                                        float (&hs)[9])
{
    float r = 0.0f;
#pragma unroll
    for (int i = 0; i < 9; ++i)
        r += dl[i];
    const bool solid = !(eps > 0.0f);
    const float ie = solid ? 0.0f : __builtin_amdgcn_rcpf(eps);
    const float om = ph.omega;
    const float base_eq = -1.5f * ie * (ux * ux + uy * uy);
    const float base_f = -3.0f * ie * (ux * Fx + uy * Fy);
    const float cg = ph.guo;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const float eu = ex_of(i) * ux + ey_of(i) * uy;
        const float eF = ex_of(i) * Fx + ey_of(i) * Fy;
        const float geq = 3.0f * eu + 4.5f * ie * eu * eu + base_eq;
        const float gf = cg * (3.0f * eF + 9.0f * ie * eu * eF + base_f);
        hs[i] = (1.0f - om) * dl[i] + w_of(i) * (om * r + rho * (om * geq + gf));
    }
}

} // namespace lbk
