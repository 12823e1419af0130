// lbk_adjoint.hip -- reverse-mode (discrete adjoint) sweep of the Klinkenberg
// lattice Boltzmann step, for gradients of a scalar read-out J of the state
// after N steps with respect to the log-permeability field ln k(x) and,
// optionally, the log base-Knudsen field ln kn0(x).
//
// The forward step n is  f^n = B(P(S_{n-1})),  S_n = C(f^n; ln k)  with P the
// pull (a permutation, bounce-back included), B the pressure-column override
// and C the per-node BGK/Guo collide (Eqs. 12, 14, 15, 17, 8, 3, 6-7).
// Given mu_n = dJ/dS_n, one reverse step computes
//   lam_f(x) = (dC/df)(x)^T mu_n(x)          (local, 9 -> 9)
//   grad(x) += (dC/d ln k)(x)^T mu_n(x)
//   mu_{n-1} = P^T B^T lam_f                 (the push: each source slot of
//                                             S_{n-1} has exactly one reader)
// C depends on f only through rho = sum f and j = sum f e, so
//   lam_f_k = (1 - omega) mu_k + G_rho + e_k . G_j
// with G_rho, G_j the total derivatives of Psi = sum_i mu_i (omega f^eq_i + F_i)
// through u(rho, j, ln k), F = -A u - B |u| u + eps G (Eq. 2; B = 0 without
// the Forchheimer term), A = eps nu / (k f_c(Kn)) and
// Kn = kn0 rho_ref / rho (so dA/d ln k = -A and dA/d ln kn0 =
// -A Kn f_c'(Kn) / f_c, which varies with rho from step to step and needs a
// gradient plane of its own); the linearisation point (rho, j) of every step is
// the history written by the recomputing forward sweep.  The read-out of J
// (global permeability or outlet flux) is the same local map with Psi the
// node's share of J and no (1 - omega) mu term.
//
// Pressure columns: the boundary node's populations are a function of its
// neighbour's (non-equilibrium extrapolation), so the thread of the
// neighbouring column also carries the boundary node's adjoint and adds
// B^T to its own; boundary threads only clear the adjoint slots whose
// forward values were discarded.
//
// Layouts (row blocks, `pitch` elements per slot, FP32): adjoint state
// [y][9][pitch]; history [y][pitch][3] = (rho, jx, jy) per node; gradient
// [y][pitch] (one plane per parameter field) accumulated in FP32 over one
// recomputed segment (at most a few hundred steps) and folded into an FP64
// total at the segment's end.  The
// adjoint state and the history are each read once, so they stream
// nontemporally.  With the Forchheimer term on, the quadratic velocity solve
// of Eq. 2 is differentiated as well (template flag FC; without it the
// Darcy path alone is compiled).
#include "lbk_adjoint.h"
#include "lbk_kernels.h"

namespace lbk {

namespace {

__device__ __forceinline__ int xcd_remap_a(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int j = b & 7, idx = b >> 3;
    return j * q + (j < r ? j : r) + idx;
}

// Forward quantities of one node's velocity solve, as in velocity() of the
// sweep, plus what the adjoint needs: dA/drho through the local Kn and
// dA/d ln kn0.
struct NodeFwd {
    float rho, rinv, jx, jy, eps, ie, A, B, c0, g, ux, uy, un, Fx, Fy, dA_drho, dA_dlnkn;
    bool solid;
};

// FC: the Forchheimer term may be on (else it is known to be off, and the
// Darcy path alone is compiled: fewer registers for the common case).
template <bool FC>
__device__ __forceinline__ NodeFwd node_fwd(const Physics &ph, float rho, float jx, float jy,
                                            float eps, float drag, float kn0)
{
    NodeFwd n;
    n.rho = rho;
    n.jx = jx;
    n.jy = jy;
    n.eps = eps;
    n.solid = !(eps > 0.0f);
    // hardware reciprocals, as in the sweep's velocity solve
    n.ie = n.solid ? 0.0f : __builtin_amdgcn_rcpf(eps);
    n.rinv = __builtin_amdgcn_rcpf(rho);
    const float kn = ph.kn_local ? kn0 * (ph.rho_ref * n.rinv) : kn0;
    float t = 0.0f; // Kn^0.4348 of the second-order correlation, once
    if (ph.corr == CORR_BKC)
        t = fc_pow(kn);
    float num, den; // f_c = den / num, as in the sweep
    fc_parts_t(ph, kn, t, num, den);
    const float dn = drag * num;
    n.A = dn * __builtin_amdgcn_rcpf(den);   // drag / f_c
    n.c0 = 1.0f + 0.5f * n.A;
    const float vx = jx * n.rinv + 0.5f * eps * ph.gx;
    const float vy = jy * n.rinv + 0.5f * eps * ph.gy;
    n.B = 0.0f;
    if (!FC || ph.feps == 0.0f) {
        const float R2 = 2.0f * __builtin_amdgcn_rcpf(2.0f * den + dn);
        n.g = den * R2; // 1 / (1 + A/2)
    } else {
        // Forchheimer (Eq. 2): c0 u + (B/2) |u| u = v, B = eps F_eps / sqrt(k_a),
        // the positive root as in the forward velocity solve
        n.B = ph.feps * __builtin_sqrtf(eps * n.A * ph.inv_nu);
        const float wn = __builtin_sqrtf(vx * vx + vy * vy);
        n.g = 2.0f / (n.c0 + __builtin_sqrtf(n.c0 * n.c0 + 2.0f * n.B * wn));
    }
    n.ux = n.solid ? 0.0f : n.g * vx;
    n.uy = n.solid ? 0.0f : n.g * vy;
    n.un = (!FC || ph.feps == 0.0f) ? 0.0f : __builtin_sqrtf(n.ux * n.ux + n.uy * n.uy);
    n.Fx = n.solid ? -2.0f * jx * n.rinv : eps * ph.gx - n.A * n.ux - n.B * n.un * n.ux;
    n.Fy = n.solid ? -2.0f * jy * n.rinv : eps * ph.gy - n.A * n.uy - n.B * n.un * n.uy;
    // Kn ~ kn0: dA/d ln kn0 = -A Kn f_c'(Kn) / f_c; with the local Kn ~ 1/rho
    // also dA/drho = -(dA/d ln kn0) / rho.  For Eqs. 6-7, f_c = P1 P2 with
    // P1 = 1 + alpha Kn = p1/a, p1 = a + 1.358 t Kn, and P2 = p2/q,
    // p2 = 1 + (4 - b) Kn, q = 1 - b Kn: P1' = 1.358 t (t + 1.4348 * 0.170)/a^2
    // and P2' = 4/q^2, so f_c'/f_c = P1'/P1 + P2'/P2
    // = 1.358 t (t + 0.243916)/(a p1) + 4/(q p2).  For Eqs. 4-5,
    // Kn f_c'/f_c = 4 Kn / (1 + 4 Kn).
    float dAk = 0.0f;
    if (kn > 0.0f && ph.corr == CORR_BKC) {
        const float a = t + 0.170f;
        const float q = 1.0f + ph.slip_nb * kn;
        const float p1 = a + 1.358f * t * kn, p2 = 1.0f + ph.slip_c * kn;
        const float l1 = 1.358f * t * (t + 0.243916f) * __builtin_amdgcn_rcpf(a * p1);
        const float l2 = 4.0f * __builtin_amdgcn_rcpf(q * p2);
        dAk = -n.A * kn * (l1 + l2);
    } else if (kn > 0.0f && ph.corr == CORR_KLINKENBERG) {
        dAk = -n.A * 4.0f * kn * __builtin_amdgcn_rcpf(1.0f + 4.0f * kn);
    }
    n.dA_dlnkn = dAk;
    n.dA_drho = ph.kn_local ? -dAk * n.rinv : 0.0f;
    return n;
}

// w-weighted moments of a 9-vector: L0 = sum w l, L1 = sum w l e,
// L2 = sum w l e e (symmetric; xx, yy, xy), from the sums and differences
// of opposite directions, each weight class applied once.
struct Mom {
    float m0, m1x, m1y, mxx, myy, mxy;
};
__device__ __forceinline__ Mom moments(const float (&l)[9])
{
    // e_5 = (1, 1), e_6 = (-1, 1), e_7 = (-1, -1), e_8 = (1, -1)
    const float a13 = l[1] + l[3], d13 = l[1] - l[3];
    const float a24 = l[2] + l[4], d24 = l[2] - l[4];
    const float a57 = l[5] + l[7], d57 = l[5] - l[7];
    const float a68 = l[6] + l[8], d68 = l[6] - l[8];
    const float sd = a57 + a68;
    const float w0 = w_of(0), w1 = w_of(1), w2 = w_of(5);
    Mom m;
    m.m0 = w0 * l[0] + w1 * (a13 + a24) + w2 * sd;
    m.m1x = w1 * d13 + w2 * (d57 - d68);
    m.m1y = w1 * d24 + w2 * (d57 + d68);
    m.mxx = w1 * a13 + w2 * sd;
    m.myy = w1 * a24 + w2 * sd;
    m.mxy = w2 * (a57 - a68);
    return m;
}

// out_i = k v_i + c + e_i . (gx, gy) for the nine directions (v = NULL: k
// v_i left out), the direction-class sums formed once.
template <bool V>
__device__ __forceinline__ void spread(float k, const float *v, float c, float gx, float gy,
                                       float (&out)[9])
{
    const float px = c + gx, mx = c - gx;
    const float t[9] = {c, px, c + gy, mx, c - gy, px + gy, mx + gy, mx - gy, px - gy};
#pragma unroll
    for (int i = 0; i < 9; ++i)
        out[i] = V ? k * v[i] + t[i] : t[i];
}

// Chain rule from the partials of a node function Psi(rho, u, F) (explicit
// Psi_rho, vectors Psi_u, Psi_F) to its total derivatives with respect to
// rho, j and ln k through the node's velocity solve.
struct Grads {
    float rho, jx, jy, lnk, lnkn;
};
__device__ __forceinline__ Grads chain(const NodeFwd &n, float Pr, float Pux, float Puy,
                                       float PFx, float PFy)
{
    Grads G;
    if (n.solid) {
        // u = 0, F = -2 j / rho
        G.jx = -2.0f * n.rinv * PFx;
        G.jy = -2.0f * n.rinv * PFy;
        G.rho = Pr + 2.0f * n.rinv * n.rinv * (PFx * n.jx + PFy * n.jy);
        G.lnk = 0.0f;
        G.lnkn = 0.0f;
        return G;
    }
    // The velocity solves M(u) = c0 u + (B/2) |u| u = v, v = j / rho + eps G / 2,
    // c0 = 1 + A/2, and F = eps G - A u - B |u| u.  With T = dPsi/du through
    // u and F(u) at fixed A, B, and K = dM/du = a I + (B/2) u u^T / |u|,
    // a = c0 + B |u| / 2: dPsi/dv = S = K^-1 T, dPsi/dj = S / rho, and
    // dPsi/dA = -(S.u / 2 + Psi_F.u) = GA, dPsi/dB = |u| GA.  B ~ sqrt(A), so
    // the B path adds GA |u| B / (2 A) per unit of dA.  Darcy (B = 0): S = T / c0.
    const float PFu = PFx * n.ux + PFy * n.uy;
    float Tx = Pux - n.A * PFx, Ty = Puy - n.A * PFy;
    float Sx, Sy, fac = 1.0f;
    if (n.B == 0.0f) {
        Sx = n.g * Tx;
        Sy = n.g * Ty;
    } else {
        const float un = n.un, hb = 0.5f * n.B * un;
        const float q = un > 0.0f ? PFu * __builtin_amdgcn_rcpf(un) : 0.0f; // u.Psi_F / |u|
        Tx -= n.B * (un * PFx + q * n.ux);
        Ty -= n.B * (un * PFy + q * n.uy);
        const float a = n.c0 + hb;
        // K^-1 = (I - b/(a + b) u u^T / |u|^2) / a with b = B |u| / 2
        const float kap =
            un > 0.0f ? 0.5f * n.B * __builtin_amdgcn_rcpf((a + hb) * un) : 0.0f;
        const float uT = n.ux * Tx + n.uy * Ty, ia = __builtin_amdgcn_rcpf(a);
        Sx = ia * (Tx - kap * uT * n.ux);
        Sy = ia * (Ty - kap * uT * n.uy);
        fac = n.A > 0.0f ? 1.0f + un * n.B * __builtin_amdgcn_rcpf(2.0f * n.A) : 1.0f;
    }
    const float GA = (-0.5f * (Sx * n.ux + Sy * n.uy) - PFu) * fac;
    G.jx = n.rinv * Sx;
    G.jy = n.rinv * Sy;
    G.rho = Pr - (G.jx * n.jx + G.jy * n.jy) * n.rinv + GA * n.dA_drho;
    G.lnk = -n.A * GA; // dA / d ln k = -A
    G.lnkn = n.dA_dlnkn * GA;
    return G;
}

// Adjoint of the collide at one node: lam_f from mu (the adjoint of the
// post-collision populations) and the sensitivity to ln k.
__device__ __forceinline__ Grads collide_adj(const Physics &ph, const NodeFwd &n,
                                             const float (&mu)[9], float (&lf)[9])
{
    const Mom L = moments(mu);
    const float om = ph.omega, cg = ph.guo, ie = n.ie;
    const float ux = n.ux, uy = n.uy, Fx = n.Fx, Fy = n.Fy;
    const float L2ux = L.mxx * ux + L.mxy * uy, L2uy = L.mxy * ux + L.myy * uy;
    const float L2Fx = L.mxx * Fx + L.mxy * Fy, L2Fy = L.mxy * Fx + L.myy * Fy;
    const float uu = ux * ux + uy * uy, uF = ux * Fx + uy * Fy;
    const float L1u = L.m1x * ux + L.m1y * uy, L1F = L.m1x * Fx + L.m1y * Fy;
    // Psi = rho { omega [L0 + 3 L1.u + 4.5/eps u.L2.u - 1.5/eps |u|^2 L0]
    //           + g [3 L1.F + 9/eps u.L2.F - 3/eps (u.F) L0] }
    const float Peq = L.m0 + 3.0f * L1u + 4.5f * ie * (ux * L2ux + uy * L2uy) - 1.5f * ie * uu * L.m0;
    const float Pf = 3.0f * L1F + 9.0f * ie * (ux * L2Fx + uy * L2Fy) - 3.0f * ie * uF * L.m0;
    const float Pr = om * Peq + cg * Pf; // Psi / rho
    const float rho = n.rho;
    const float Pux = rho * (om * (3.0f * L.m1x + 9.0f * ie * L2ux - 3.0f * ie * L.m0 * ux) +
                             cg * (9.0f * ie * L2Fx - 3.0f * ie * L.m0 * Fx));
    const float Puy = rho * (om * (3.0f * L.m1y + 9.0f * ie * L2uy - 3.0f * ie * L.m0 * uy) +
                             cg * (9.0f * ie * L2Fy - 3.0f * ie * L.m0 * Fy));
    const float PFx = rho * cg * (3.0f * L.m1x + 9.0f * ie * L2ux - 3.0f * ie * L.m0 * ux);
    const float PFy = rho * cg * (3.0f * L.m1y + 9.0f * ie * L2uy - 3.0f * ie * L.m0 * uy);
    const Grads G = chain(n, Pr, Pux, Puy, PFx, PFy);
    spread<true>(1.0f - om, mu, G.rho, G.jx, G.jy, lf);
    return G;
}

// Adjoint of the read-out share of J at one node, J_x = a1 rho u_x + a2 u_x.
__device__ __forceinline__ Grads readout_adj(const NodeFwd &n, float a1, float a2,
                                             float (&lf)[9])
{
    Grads G{0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (!n.solid && (a1 != 0.0f || a2 != 0.0f))
        G = chain(n, a1 * n.ux, a1 * n.rho + a2, 0.0f, 0.0f, 0.0f);
    spread<false>(0.0f, nullptr, G.rho, G.jx, G.jy, lf);
    return G;
}

// Adjoint of the pressure-column override
//   f_i(b) = f_eq_i(rho_b, u_n; eps_b) + f_i(n) - f_eq_i(rho_n, u_n; eps_n)
// with respect to the neighbour's post-stream populations f(n) (through
// f(n) itself, rho_n, j_n and u_n(rho_n, j_n, ln k_n)).  Adds to lfn and
// returns the neighbour's ln k and ln kn0 sensitivities.
__device__ __forceinline__ float2 nee_adj(const NodeFwd &n, float rho_b, float eps_b,
                                         const float (&lb)[9], float (&lfn)[9])
{
    const Mom M = moments(lb);
    const float ux = n.ux, uy = n.uy;
    const float M2ux = M.mxx * ux + M.mxy * uy, M2uy = M.mxy * ux + M.myy * uy;
    const float uu = ux * ux + uy * uy;
    // Phi(rho, eps) = sum_i lb_i f_eq_i = rho [M0 + 3 M1.u + 4.5/eps u.M2.u
    //                 - 1.5/eps |u|^2 M0]; for eps = 0 it is rho M0.
    const bool sb = !(eps_b > 0.0f);
    const float ieb = sb ? 0.0f : __builtin_amdgcn_rcpf(eps_b), ien = n.ie;
    const float dbx = sb ? 0.0f : rho_b * (3.0f * M.m1x + 9.0f * ieb * M2ux - 3.0f * ieb * M.m0 * ux);
    const float dby = sb ? 0.0f : rho_b * (3.0f * M.m1y + 9.0f * ieb * M2uy - 3.0f * ieb * M.m0 * uy);
    const float dnx = n.solid ? 0.0f : n.rho * (3.0f * M.m1x + 9.0f * ien * M2ux - 3.0f * ien * M.m0 * ux);
    const float dny = n.solid ? 0.0f : n.rho * (3.0f * M.m1y + 9.0f * ien * M2uy - 3.0f * ien * M.m0 * uy);
    const float phin_over_rho =
        n.solid ? M.m0
                : M.m0 + 3.0f * (M.m1x * ux + M.m1y * uy) + 4.5f * ien * (ux * M2ux + uy * M2uy) -
                      1.5f * ien * uu * M.m0;
    // Psi = Phi_b(u) - Phi_n(rho_n, u): explicit d/drho_n = -Phi_n / rho_n,
    // d/du = Hu; no direct force dependence.
    const Grads G = chain(n, -phin_over_rho, dbx - dnx, dby - dny, 0.0f, 0.0f);
    float gx = G.jx, gy = G.jy, gr = G.rho, gl = G.lnk, gk = G.lnkn;
    if (n.solid) { // u_n = 0 does not move with f(n)
        gx = gy = gl = gk = 0.0f;
        gr = -phin_over_rho;
    }
    float add[9];
    spread<true>(1.0f, lb, gr, gx, gy, add);
#pragma unroll
    for (int i = 0; i < 9; ++i)
        lfn[i] += add[i];
    return make_float2(gl, gk);
}

__device__ __forceinline__ Rsrc rsrc_row(const void *base, uint64_t row_bytes, int y)
{
    return make_rsrc(static_cast<const char *>(base) + (uint64_t)y * row_bytes,
                     (uint32_t)row_bytes);
}

} // namespace

// One reverse step (or, with terminal != 0, the read-out of J).
//   mu_in  [y][9][pitch]  adjoint of S_n (ignored when terminal)
//   mu_out [y][9][pitch]  adjoint of S_{n-1} (written by push)
//   hist   [y][pitch][3]  (rho, jx, jy) of step n's post-stream populations
//   grad   [y][pitch]     FP32, accumulates d J / d ln k over a segment
//   grad2  [y][pitch]     FP32, d J / d ln kn0 likewise (KN only)
// Objective: J = sum_x a1(x) rho u_x + a2 u_x with a1(x) = a1 (all nodes,
// or only column nx-1 when outlet != 0) and a2 uniform.
template <int BCX, int BCY, bool KN, bool FC>
__device__ __forceinline__ void adjoint_node(const float *mu_in, float *mu_out, const float *hist,
                                             const char *med, const MLayout &mlay, float *grad,
                                             float *grad2, const Geom &g, const Physics &ph,
                                             int terminal, float a1, float a2, int outlet, int y,
                                             uint32_t x)
{
    const uint32_t nx = (uint32_t)g.nx;
    const uint64_t lrow = 9ull * g.pitch * 4, hrow = 3ull * g.pitch * 4;
    const uint32_t slot = (uint32_t)g.pitch * 4; // bytes per FP32 slot
    const Rsrc hr = rsrc_row(hist, hrow, y);
    const Rsrc mr = make_rsrc(med + (uint64_t)y * mlay.row, (uint32_t)mlay.row);
    const Rsrc lin = rsrc_row(mu_in, lrow, y);
    float *grow_p = grad + (uint64_t)y * g.pitch;
    float *grow_k = KN ? grad2 + (uint64_t)y * g.pitch : nullptr;

    auto load_node = [&](uint32_t xx) {
        float h[3];
        ld_hist<kNT>(hr, xx * 12, h);
        return node_fwd<FC>(ph, h[0], h[1], h[2], ld_f32(mr, xx * 4, 0),
                            ld_f32(mr, xx * 4, mlay.slot), ld_f32(mr, xx * 4, 2 * mlay.slot));
    };
    auto node_adj = [&](const NodeFwd &n, uint32_t xx, float (&lf)[9]) {
        if (terminal) {
            const float a = (!outlet || xx == nx - 1) ? a1 : 0.0f;
            return readout_adj(n, a, a2, lf);
        }
        float mu[9];
#pragma unroll
        for (int i = 0; i < 9; ++i)
            mu[i] = ld_f32_nt(lin, xx * 4, i * slot);
        return collide_adj(ph, n, mu, lf);
    };
    // each gradient entry has exactly one writer per launch
    auto add_grad = [&](uint32_t xx, float v, float vk) {
        grow_p[xx] += v;
        if (KN)
            grow_k[xx] += vk;
    };

    // rows the push writes into: source of direction i is (x - e_ix, y - e_iy)
    int ym = y - 1, yp = y + 1;
    bool wym = false, wyp = false;
    if (BCY == BC_PERIODIC) {
        ym = (y == 0) ? g.ny - 1 : ym;
        yp = (y == g.ny - 1) ? 0 : yp;
    } else {
        // scalar wall flags (the row is the workgroup's): keeps the selects
        // of the pushed rows' buffer resources scalar
        wym = __builtin_amdgcn_readfirstlane(y == 0 ? 1 : 0) != 0;
        wyp = __builtin_amdgcn_readfirstlane(y == g.ny - 1 ? 1 : 0) != 0;
        ym = wym ? y : ym;
        yp = wyp ? y : yp;
    }
    const Rsrc orow[3] = {rsrc_row(mu_out, lrow, ym), rsrc_row(mu_out, lrow, y),
                          rsrc_row(mu_out, lrow, yp)};

    float lf[9];
    const bool bnode = (BCX == BC_PRESSURE) && (x == 0 || x == nx - 1);
    if (bnode) {
        // forward values pulled into this node were discarded: clear the
        // slots it would push to, and the slots whose destination lies
        // outside the lattice
#pragma unroll
        for (int i = 0; i < 9; ++i)
            lf[i] = 0.0f;
    } else {
        const NodeFwd n = load_node(x);
        const Grads G = node_adj(n, x, lf);
        float gl = G.lnk, gk = G.lnkn;
        if (BCX == BC_PRESSURE && (x == 1 || x == nx - 2)) {
            // carry the boundary node next door (x = 0 or nx-1)
            const uint32_t xb = (x == 1) ? 0 : nx - 1;
            {
                const NodeFwd b = load_node(xb);
                float lb[9];
                const Grads Gb = node_adj(b, xb, lb);
                add_grad(xb, Gb.lnk, Gb.lnkn);
                const float2 gn = nee_adj(n, b.rho, b.eps, lb, lf);
                gl += gn.x;
                gk += gn.y;
            }
            if (nx == 3) {
                // x = 1 is the neighbour of both columns: the outlet too
                const NodeFwd b = load_node(2);
                float lb[9];
                const Grads Gb = node_adj(b, 2, lb);
                add_grad(2, Gb.lnk, Gb.lnkn);
                const float2 gn = nee_adj(n, b.rho, b.eps, lb, lf);
                gl += gn.x;
                gk += gn.y;
            }
        }
        add_grad(x, gl, gk);
    }

    // push: mu_out[i](x - e_i) = lf_i, bounce-back at walls.  The pushed
    // stores keep the default cache policy: a wave's shifted store covers
    // parts of two cache lines whose other parts the neighbouring wave
    // writes, and L2 merges them (3% less gradient time than streaming
    // stores on the 8192^2 shale)
    uint32_t xm = x - 1, xp = x + 1;
    bool wxm = false, wxp = false;
    if (BCX == BC_PERIODIC) {
        xm = (x == 0) ? nx - 1 : xm;
        xp = (x == nx - 1) ? 0 : xp;
    } else if (BCX == BC_WALL) {
        wxm = (x == 0);
        wxp = (x == nx - 1);
    } else {
        wxm = (x == 0); // pressure: nothing beyond the end columns
        wxp = (x == nx - 1);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int ex = ex_of(i), ey = ey_of(i);
        const bool wall_y = (ey == 1 && wym) || (ey == -1 && wyp); // uniform
        const bool out_x = (ex == 1 && wxm) || (ex == -1 && wxp);  // per lane
        const int ry = ey == 1 ? 0 : (ey == -1 ? 2 : 1);
        const uint32_t tx = ex == 1 ? xm : (ex == -1 ? xp : x);
        if (BCX == BC_PRESSURE) {
            if (out_x)
                continue; // source outside the lattice
            if (wall_y)
                st_f32(orow[1], x * 4, opp_of(i) * slot, lf[i], false);
            else
                st_f32(orow[ry], tx * 4, i * slot, lf[i], false);
        } else {
            if (wall_y || out_x)
                st_f32(orow[1], x * 4, opp_of(i) * slot, lf[i], false);
            else
                st_f32(orow[ry], tx * 4, i * slot, lf[i], false);
        }
    }
    if (BCX == BC_PRESSURE && bnode) {
        // slots of this node whose forward destination lies outside
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const int ex = ex_of(i);
            if ((x == 0 && ex == -1) || (x == nx - 1 && ex == 1))
                st_f32(orow[1], x * 4, i * slot, 0.0f, false);
        }
    }
}

template <int BCX, int BCY, bool KN, bool FC>
__global__ __launch_bounds__(256) void adjoint_kernel(const float *mu_in, float *mu_out,
                                                       const float *hist, const char *med,
                                                       MLayout mlay, float *grad, float *grad2,
                                                       Geom g, Physics ph, int terminal,
                                                       float a1, float a2, int outlet, int bpr)
{
    const int L = xcd_remap_a(blockIdx.x, gridDim.x);
    const int y = L / bpr;
    const uint32_t x = (uint32_t)(L - y * bpr) * 256 + threadIdx.x;
    if (x >= (uint32_t)g.nx)
        return;
    adjoint_node<BCX, BCY, KN, FC>(mu_in, mu_out, hist, med, mlay, grad, grad2, g, ph, terminal, a1,
                               a2, outlet, y, x);
}

// ------------------------------------------------ two reverse steps per pass
//
// adjoint2_kernel takes mu_n to mu_{n-2} in one pass, bitwise what two
// adjoint_kernel launches through mu_{n-1} give, with mu_{n-1} never
// leaving registers.  In gather form a reverse step reads
//   mu_{n-1}(x, j) = lam_f_j(x + e_j),
// lam_f_{opp j}(x) where x + e_j lies beyond a wall (bounce-back), and 0
// where x + e_j lies beyond a pressure column; lam_f itself is local to its
// node (plus, at the column next to a pressure column, that column's
// contribution through the non-equilibrium extrapolation).  As in the
// forward two-step pass, a wave holds a strip of 64 columns (60 of its own
// and two halo columns on either side, x neighbours through DPP lane shifts)
// and marches down a band of rows; lam_f of step n, mu_{n-1} and lam_f of
// step n-1 of the rows around the current one stay in registers, and each
// gradient entry collects both steps' terms before it is written once.
namespace {

// Lane-dependent facts of a strip of the reverse pass.
struct ALanes {
    uint32_t x;         // the lane's column, wrapped (periodic) or clamped
    bool wxm, wxp;      // wall x: the column is the first / last
    bool first, last;   // pressure x: the inlet / outlet column
    bool cl, cr;        // pressure x: the column next to the inlet / outlet
    bool has_b;         // uniform: the wave may hold any of these
    bool bgrad;         // pressure columns receive gradient terms (nx >= 3)
};

// A row's inputs at this lane's column, in two parts loaded at different
// times: what the reverse of step n needs (mu_n, the history of step n and
// the medium) and what the reverse of step n - 1 adds (the history of step
// n - 1 and the medium again).  Each part is loaded straight into the
// registers where it is used, and nothing loaded is copied to another
// register, so no load is waited for before its use.
struct RowA {
    float mu[9], h1[3], md[3];
};
struct RowB {
    float h0[3], md[3];
};
// After the reverse of step n, and after that of step n - 1: lam_f and the
// gradient terms.
struct AMid {
    float lf[9], gl, gk;
};

// lam_f and the ln k / ln kn0 terms of one reverse step at this lane's node
// (adjoint_node's arithmetic, with a pressure column's contribution taken
// from the neighbouring lane rather than recomputed).
template <int BCX, bool FC>
__device__ __forceinline__ void local_adj(const Physics &ph, const float (&mu)[9], const float (&h)[3],
                                          const float (&md)[3], const ALanes &ln,
                                          float (&lf)[9], float &gl, float &gk)
{
    const NodeFwd n = node_fwd<FC>(ph, h[0], h[1], h[2], md[0], md[1], md[2]);
    const Grads G = collide_adj(ph, n, mu, lf);
    gl = G.lnk;
    gk = G.lnkn;
    if (BCX != BC_PRESSURE)
        return;
    if (ln.has_b) {
        // the pressure columns' lam_f as computed so far (never changed by
        // the carries below, which only touch the columns next to them)
        float lb[9];
#pragma unroll
        for (int i = 0; i < 9; ++i)
            lb[i] = lane_from<1>(lf[i]);
        float rb = lane_from<1>(n.rho), eb = lane_from<1>(n.eps);
        if (ln.cl) {
            const float2 q = nee_adj(n, rb, eb, lb, lf);
            gl += q.x;
            gk += q.y;
        }
#pragma unroll
        for (int i = 0; i < 9; ++i)
            lb[i] = lane_from<-1>(lf[i]);
        rb = lane_from<-1>(n.rho);
        eb = lane_from<-1>(n.eps);
        if (ln.cr) {
            const float2 q = nee_adj(n, rb, eb, lb, lf);
            gl += q.x;
            gk += q.y;
        }
    }
    if (ln.first || ln.last) {
        // forward values pulled into a pressure column are discarded
#pragma unroll
        for (int i = 0; i < 9; ++i)
            lf[i] = 0.0f;
        if (!ln.bgrad)
            gl = gk = 0.0f;
    }
}

// mu of this lane's node from lam_f of rows y - 1 (dn), y (c), y + 1 (up).
// wym / wyp: the row below / above lies beyond a wall.
template <int BCX>
__device__ __forceinline__ void gather(const float (&dn)[9], const float (&c)[9],
                                       const float (&up)[9], bool wym, bool wyp,
                                       const ALanes &ln, float (&mu)[9])
{
    mu[0] = c[0];
#pragma unroll
    for (int j = 1; j < 9; ++j) {
        const int ex = ex_of(j), ey = ey_of(j);
        const bool wall_y = (ey == 1 && wyp) || (ey == -1 && wym); // uniform
        const float(&r)[9] = ey == 1 ? up : (ey == -1 ? dn : c);
        float v;
        if (wall_y)
            v = c[opp_of(j)];
        else if (ex == 1)
            v = lane_from<-1>(r[j]);
        else if (ex == -1)
            v = lane_from<1>(r[j]);
        else
            v = r[j];
        if (BCX == BC_WALL) {
            const bool out_x = (ex == 1 && ln.wxp) || (ex == -1 && ln.wxm);
            if (out_x)
                v = c[opp_of(j)];
        }
        if (BCX == BC_PRESSURE) {
            const bool out_x = (ex == 1 && ln.last) || (ex == -1 && ln.first);
            if (out_x)
                v = 0.0f;
        }
        mu[j] = v;
    }
}

} // namespace

// Two reverse steps: mu_in = mu_n -> mu_out = mu_{n-2}, hist1 / hist0 the
// histories of steps n and n - 1, grad / grad2 as in adjoint_node.  Rows
// are marched in bands of `band`; a block holds four strips.
// The pass of one wave: strip `strip` of band `bnd` of one lattice.
template <int BCX, int BCY, bool KN, bool FC>
__device__ __forceinline__ void adjoint2_strip(
    const float *__restrict__ mu_in, float *__restrict__ mu_out, const float *__restrict__ hist1,
    const float *__restrict__ hist0, const char *__restrict__ med, const MLayout &mlay,
    float *__restrict__ grad, float *__restrict__ grad2, const Geom &g, const Physics &ph,
    int band, int bnd, int strip)
{
    const int lane = (int)(threadIdx.x & 63);
    const int nx = g.nx, ny = g.ny;
    const int nstrips = (nx + kStrip2 - 1) / kStrip2;
    if (strip >= nstrips)
        return; // the whole wave
    // Strip s owns columns [c0, c1).  With pressure columns the last strip
    // starts at most at nx - 4: the column next to the outlet then never
    // sits at lane 63 of a strip that owns the column two to its left, whose
    // result would need the outlet column's values from beyond the wave.
    int c0 = strip * kStrip2, c1 = min(c0 + kStrip2, nx);
    if (BCX == BC_PRESSURE) {
        const int cl = max(0, min(kStrip2 * (nstrips - 1), nx - 4));
        if (strip == nstrips - 1)
            c0 = cl;
        else if (strip == nstrips - 2)
            c1 = cl;
    }
    const int xr = c0 - 2 + lane;
    const bool owned = xr >= c0 && xr < c1;
    ALanes ln;
    if (BCX == BC_PERIODIC)
        ln.x = (uint32_t)(((xr % nx) + nx) % nx);
    else
        ln.x = (uint32_t)(xr < 0 ? 0 : (xr >= nx ? nx - 1 : xr)); // beyond: unused copies
    ln.wxm = BCX == BC_WALL && xr == 0;
    ln.wxp = BCX == BC_WALL && xr == nx - 1;
    ln.first = BCX == BC_PRESSURE && xr == 0;
    ln.last = BCX == BC_PRESSURE && xr == nx - 1;
    ln.cl = BCX == BC_PRESSURE && nx >= 3 && xr == 1;
    ln.cr = BCX == BC_PRESSURE && nx >= 3 && xr == nx - 2;
    ln.has_b = BCX == BC_PRESSURE && (strip == 0 || strip >= nstrips - 2);
    ln.bgrad = nx >= 3;
    const int y0 = bnd * band, y1 = min(y0 + band, ny);
    auto exists = [&](int y) { return BCY == BC_PERIODIC || (y >= 0 && y < ny); };
    auto wrap = [&](int y) { return BCY == BC_PERIODIC ? ((y % ny) + ny) % ny : y; };
    // a row that always exists (beyond a wall: the nearest row, loaded but
    // never used, since the gather bounces back there)
    auto held = [&](int y) {
        return BCY == BC_PERIODIC ? wrap(y) : (y < 0 ? 0 : (y >= ny ? ny - 1 : y));
    };
    auto wall_lo = [&](int y) { return BCY == BC_WALL && y == 0; };
    auto wall_hi = [&](int y) { return BCY == BC_WALL && y == ny - 1; };
    // Unconditional stores (see sweep2_kernel): a lane that does not own
    // its column repeats the store of the wave's first owning lane.
    const uint64_t om = __builtin_amdgcn_ballot_w64(owned);
    if (om == 0)
        return;
    const int q = (int)__builtin_ctzll(om);
    const uint32_t xq = (uint32_t)__builtin_amdgcn_readlane((int)ln.x, q);
    const uint32_t xst = owned ? ln.x : xq;
    auto same = [&](float v) {
        const float vq = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), q));
        return owned ? v : vq;
    };

    const uint64_t lrow = 9ull * g.pitch * 4, hrow = 3ull * g.pitch * 4;
    const uint64_t grow = (uint64_t)g.pitch * 4;
    const uint32_t slot = (uint32_t)g.pitch * 4;
    const uint32_t xo = ln.x * 4;
    // Loads keep the default cache policy: a strip's first and last cache
    // lines are shared with the neighbouring strips, which read them about
    // the same time.
    // The march loads ahead of its needs; rows past them (first parts
    // beyond y1 + 1, second parts beyond y1: the last output row's) get
    // empty buffer resources, so their loads return 0 without touching
    // memory.
    auto row_of = [&](const void *base, uint64_t bytes, int yh, bool live) {
        return make_rsrc(static_cast<const char *>(base) + (uint64_t)yh * bytes,
                         live ? (uint32_t)bytes : 0u);
    };
    auto load_a = [&](int y, RowA &r) {
        const int yh = held(y);
        const bool live = y <= y1 + 1;
        const Rsrc lr = row_of(mu_in, lrow, yh, live);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            r.mu[i] = ld_f32(lr, xo, i * slot);
        const Rsrc hr = row_of(hist1, hrow, yh, live), mr = row_of(med, mlay.row, yh, live);
        ld_hist<0>(hr, ln.x * 12, r.h1);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            r.md[k] = ld_f32(mr, xo, k * mlay.slot);
    };
    auto load_b = [&](int y, RowB &r) {
        const int yh = held(y);
        const bool live = y <= y1;
        const Rsrc hr = row_of(hist0, hrow, yh, live), mr = row_of(med, mlay.row, yh, live);
        ld_hist<0>(hr, ln.x * 12, r.h0);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            r.md[k] = ld_f32(mr, xo, k * mlay.slot);
    };
    auto step_a = [&](const RowA &r, AMid &a) {
        local_adj<BCX, FC>(ph, r.mu, r.h1, r.md, ln, a.lf, a.gl, a.gk);
    };
    auto step_b = [&](int y, const AMid &dn, const AMid &c, const AMid &up, const RowB &r,
                      AMid &b) {
        float mu[9];
        gather<BCX>(dn.lf, c.lf, up.lf, wall_lo(y), wall_hi(y), ln, mu);
        local_adj<BCX, FC>(ph, mu, r.h0, r.md, ln, b.lf, b.gl, b.gk);
    };
    // Output row y from lam_f of step n - 1 of rows y - 1 .. y + 1; the
    // gradient entries add the terms of step n (a) and then of step n - 1
    // (c), in the order of two single reverse steps.
    auto emit = [&](int y, const AMid &dn, const AMid &c, const AMid &up, const AMid &a,
                    float gp, float gk) {
        float mu[9];
        gather<BCX>(dn.lf, c.lf, up.lf, wall_lo(y), wall_hi(y), ln, mu);
        const Rsrc orow = rsrc_row(mu_out, lrow, y);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            st_f32(orow, xst * 4, i * slot, same(mu[i]), false);
        st_f32(rsrc_row(grad, grow, y), xst * 4, 0, same((gp + a.gl) + c.gl), false);
        if (KN)
            st_f32(rsrc_row(grad2, grow, y), xst * 4, 0, same((gk + a.gk) + c.gk), false);
    };

    // For output row y: lam_f of step n of rows y .. y + 2 (A slots), of
    // step n - 1 of rows y - 1 .. y + 1 (B slots).  The first input parts
    // of rows y + 2 .. y + 4 and the second parts of rows y + 1 .. y + 3 are
    // in flight (three slots each, reloaded as soon as consumed).
    RowA P, Q, S;
    RowB U, V, W;
    AMid A0{}, A1{}, A2{}, B0{}, B1{}, B2{};
    load_a(y0 - 2, P);
    load_a(y0 - 1, Q);
    load_a(y0, S);
    load_b(y0 - 1, U);
    load_b(y0, V);
    load_b(y0 + 2, W);
    if (exists(y0 - 2))
        step_a(P, A0);
    load_a(y0 + 1, P);
    if (exists(y0 - 1))
        step_a(Q, A1);
    load_a(y0 + 2, Q);
    step_a(S, A2);
    load_a(y0 + 3, S);
    if (exists(y0 - 1))
        step_b(wrap(y0 - 1), A0, A1, A2, U, B0);
    load_b(y0 + 1, U);
    if (exists(y0 + 1))
        step_a(P, A0);
    load_a(y0 + 4, P);
    step_b(y0, A1, A2, A0, V, B1);
    load_b(y0 + 3, V);
    // One output row y, the slots in rotated roles (period 3).
    // The gradient entries of row y are read at the start of its row, a
    // whole row's arithmetic before they are needed.
    auto row = [&](int y, RowA &ra, AMid &na, const AMid &adn, const AMid &ac, RowB &rb,
                   AMid &nb, const AMid &bdn, const AMid &bc) {
        const float gp = ld_f32(rsrc_row(grad, grow, y), xo, 0);
        const float gk = KN ? ld_f32(rsrc_row(grad2, grow, y), xo, 0) : 0.0f;
        if (exists(y + 2))
            step_a(ra, na);
        load_a(y + 5, ra);
        if (exists(y + 1))
            step_b(wrap(y + 1), adn, ac, na, rb, nb);
        load_b(y + 4, rb);
        emit(y, bdn, bc, nb, adn, gp, gk);
    };
    // Whole periods in the loop, the last one or two rows after it: a loop
    // with exits between its rows made the compiler copy loaded values at
    // the back edge, waiting there for the loads just issued.
    int y = y0;
    for (; y + 3 <= y1; y += 3) {
        row(y, Q, A1, A2, A0, U, B2, B0, B1);
        row(y + 1, S, A2, A0, A1, W, B0, B1, B2);
        row(y + 2, P, A0, A1, A2, V, B1, B2, B0);
    }
    if (y < y1) {
        row(y, Q, A1, A2, A0, U, B2, B0, B1);
        if (y + 1 < y1)
            row(y + 1, S, A2, A0, A1, W, B0, B1, B2);
    }
}

template <int BCX, int BCY, bool KN, bool FC>
__global__ __launch_bounds__(256) void adjoint2_kernel(
    const float *__restrict__ mu_in, float *__restrict__ mu_out, const float *__restrict__ hist1,
    const float *__restrict__ hist0, const char *__restrict__ med, MLayout mlay,
    float *__restrict__ grad, float *__restrict__ grad2, Geom g, Physics ph, int band, int groups)
{
    // logical block: band-major, four strips (one per wave) per block
    const int L = xcd_remap_a(blockIdx.x, gridDim.x);
    const int bnd = L / groups;
    const int strip = (L - bnd * groups) * 4 + (int)(threadIdx.x >> 6);
    adjoint2_strip<BCX, BCY, KN, FC>(mu_in, mu_out, hist1, hist0, med, mlay, grad, grad2, g, ph,
                                     band, bnd, strip);
}

// total += seg; seg = 0 (end of a recomputed segment)
__global__ __launch_bounds__(256) void grad_fold_kernel(float *seg, double *total, Geom g,
                                                         int bpr)
{
    const int L = xcd_remap_a(blockIdx.x, gridDim.x);
    const int y = L / bpr;
    const int x = (L - y * bpr) * 256 + threadIdx.x;
    if (x >= g.nx)
        return;
    const int64_t c = (int64_t)y * g.pitch + x;
    total[c] += (double)seg[c];
    seg[c] = 0.0f;
}

__global__ __launch_bounds__(256) void grad_out_kernel(const double *grad, float *out, Geom g,
                                                        int bpr)
{
    const int L = xcd_remap_a(blockIdx.x, gridDim.x);
    const int y = L / bpr;
    const int x = (L - y * bpr) * 256 + threadIdx.x;
    if (x >= g.nx)
        return;
    out[(int64_t)y * g.nx + x] = (float)grad[(int64_t)y * g.pitch + x];
}

template <int BCX, int BCY>
static hipError_t adj_t(const float *mu_in, float *mu_out, const float *hist, const char *med,
                        const MLayout &mlay, float *grad, float *grad2, const Geom &g,
                        const Physics &ph, int terminal, float a1, float a2, int outlet,
                        hipStream_t st)
{
    const int bpr = (g.nx + 255) / 256;
#define LBK_ADJK(KN, FC)                                                                     \
    hipLaunchKernelGGL((adjoint_kernel<BCX, BCY, KN, FC>), dim3(bpr * g.ny), dim3(256), 0, st, \
                       mu_in, mu_out, hist, med, mlay, grad, grad2, g, ph, terminal, a1, a2,   \
                       outlet, bpr)
    const bool fc = ph.feps != 0.0f;
    if (grad2 && fc)
        LBK_ADJK(true, true);
    else if (grad2)
        LBK_ADJK(true, false);
    else if (fc)
        LBK_ADJK(false, true);
    else
        LBK_ADJK(false, false);
#undef LBK_ADJK
    return hipGetLastError();
}

hipError_t launch_adjoint(int bcx, int bcy, const float *mu_in, float *mu_out, const float *hist,
                          const char *med, const MLayout &mlay, float *grad, float *grad2,
                          const Geom &g, const Physics &ph, int terminal, float a1, float a2,
                          int outlet, hipStream_t st)
{
#define LBK_ADJ(X, Y)                                                                        \
    adj_t<X, Y>(mu_in, mu_out, hist, med, mlay, grad, grad2, g, ph, terminal, a1, a2, outlet, st)
    switch (bcx * 2 + bcy) {
    case 0: return LBK_ADJ(BC_PERIODIC, BC_PERIODIC);
    case 1: return LBK_ADJ(BC_PERIODIC, BC_WALL);
    case 2: return LBK_ADJ(BC_WALL, BC_PERIODIC);
    case 3: return LBK_ADJ(BC_WALL, BC_WALL);
    case 4: return LBK_ADJ(BC_PRESSURE, BC_PERIODIC);
    case 5: return LBK_ADJ(BC_PRESSURE, BC_WALL);
    default: return hipErrorInvalidValue;
    }
#undef LBK_ADJ
}

template <int BCX, int BCY>
static hipError_t adj2_t(const float *mu_in, float *mu_out, const float *hist1,
                         const float *hist0, const char *med, const MLayout &mlay, float *grad,
                         float *grad2, const Geom &g, const Physics &ph, int band, hipStream_t st)
{
    const int nstrips = (g.nx + kStrip2 - 1) / kStrip2;
    const int groups = (nstrips + 3) / 4;
    const int blocks = groups * ((g.ny + band - 1) / band);
#define LBK_ADJ2K(KN, FC)                                                                    \
    hipLaunchKernelGGL((adjoint2_kernel<BCX, BCY, KN, FC>), dim3(blocks), dim3(256), 0, st,    \
                       mu_in, mu_out, hist1, hist0, med, mlay, grad, grad2, g, ph, band, groups)
    const bool fc = ph.feps != 0.0f;
    if (grad2 && fc)
        LBK_ADJ2K(true, true);
    else if (grad2)
        LBK_ADJ2K(true, false);
    else if (fc)
        LBK_ADJ2K(false, true);
    else
        LBK_ADJ2K(false, false);
#undef LBK_ADJ2K
    return hipGetLastError();
}

hipError_t launch_adjoint2(int bcx, int bcy, const float *mu_in, float *mu_out,
                           const float *hist1, const float *hist0, const char *med,
                           const MLayout &mlay, float *grad, float *grad2, const Geom &g,
                           const Physics &ph, int band, hipStream_t st)
{
    if (band < 1 || mu_in == mu_out)
        return hipErrorInvalidValue;
#define LBK_ADJ2(X, Y)                                                                       \
    adj2_t<X, Y>(mu_in, mu_out, hist1, hist0, med, mlay, grad, grad2, g, ph, band, st)
    switch (bcx * 2 + bcy) {
    case 0: return LBK_ADJ2(BC_PERIODIC, BC_PERIODIC);
    case 1: return LBK_ADJ2(BC_PERIODIC, BC_WALL);
    case 2: return LBK_ADJ2(BC_WALL, BC_PERIODIC);
    case 3: return LBK_ADJ2(BC_WALL, BC_WALL);
    case 4: return LBK_ADJ2(BC_PRESSURE, BC_PERIODIC);
    case 5: return LBK_ADJ2(BC_PRESSURE, BC_WALL);
    default: return hipErrorInvalidValue;
    }
#undef LBK_ADJ2
}

hipError_t launch_grad_fold(float *seg, double *total, const Geom &g, hipStream_t st)
{
    const int bpr = (g.nx + 255) / 256;
    hipLaunchKernelGGL(grad_fold_kernel, dim3(bpr * g.ny), dim3(256), 0, st, seg, total, g, bpr);
    return hipGetLastError();
}

hipError_t launch_grad_out(const double *grad, float *out, const Geom &g, hipStream_t st)
{
    const int bpr = (g.nx + 255) / 256;
    hipLaunchKernelGGL(grad_out_kernel, dim3(bpr * g.ny), dim3(256), 0, st, grad, out, g, bpr);
    return hipGetLastError();
}

// ------------------------------------------------------ batched gradients
//
// The same reverse step, fold and output over a batch's tile list (tiles of
// blockDim.x by rows, one workgroup per tile); each sample's regions come
// from its descriptor, copied to registers before the first store.

__device__ __forceinline__ bool adj_tile(const AdjSampleDesc *__restrict__ samples,
                                         const int *__restrict__ tile_sample, int rows,
                                         AdjSampleDesc &sd, uint32_t &x, int &y0, int &y1)
{
    const int t = xcd_remap_a(blockIdx.x, gridDim.x);
    sd = samples[tile_sample[t]];
    const int rel = t - sd.tile0;
    const int ty = rel / sd.tpr;
    x = (uint32_t)(rel - ty * sd.tpr) * blockDim.x + threadIdx.x;
    y0 = ty * rows;
    y1 = min(y0 + rows, sd.g.ny);
    return x < (uint32_t)sd.g.nx;
}

// lam_in < 0: the terminal read-out (writes lam[0]); else lam[lam_in] ->
// lam[lam_in ^ 1].  hist_slot: the history of the step being reversed.
template <int BCX, int BCY, bool KN, bool FC>
__global__ __launch_bounds__(256) void batch_adjoint_kernel(
    const AdjSampleDesc *__restrict__ samples, const int *__restrict__ tile_sample, int rows,
    int lam_in, int hist_slot)
{
    AdjSampleDesc sd;
    uint32_t x;
    int y0, y1;
    if (!adj_tile(samples, tile_sample, rows, sd, x, y0, y1))
        return;
    const bool terminal = lam_in < 0;
    const float *mu_in = terminal ? nullptr : (lam_in ? sd.lam[1] : sd.lam[0]);
    float *mu_out = terminal ? sd.lam[0] : (lam_in ? sd.lam[0] : sd.lam[1]);
    const float *hist = reinterpret_cast<const float *>(reinterpret_cast<const char *>(sd.hist) +
                                                        (uint64_t)hist_slot * sd.hist_bytes);
    for (int y = y0; y < y1; ++y)
        adjoint_node<BCX, BCY, KN, FC>(mu_in, mu_out, hist, sd.med, sd.mlay, sd.seg, sd.seg2, sd.g,
                                   sd.ph, terminal ? 1 : 0, sd.a1, sd.a2, sd.outlet, y, x);
}

// Two reverse steps of every sample, lam[lam_in] -> lam[lam_in ^ 1], the
// histories in slots hist_slot (the later step) and hist_slot - 1: tiles of
// four strips by `band` rows (the batch's two-step tiling: tile0 / tpr give
// a sample's first tile and its groups of four strips per band).
template <int BCX, int BCY, bool KN, bool FC>
__global__ __launch_bounds__(256) void batch_adjoint2_kernel(
    const AdjSampleDesc *__restrict__ samples, const int *__restrict__ tile_sample, int band,
    int lam_in, int hist_slot)
{
    const int t = xcd_remap_a(blockIdx.x, gridDim.x);
    const AdjSampleDesc sd = samples[tile_sample[t]];
    const int rel = t - sd.tile0;
    const int bnd = rel / sd.tpr;
    const int strip = (rel - bnd * sd.tpr) * 4 + (int)(threadIdx.x >> 6);
    const float *mu_in = lam_in ? sd.lam[1] : sd.lam[0];
    float *mu_out = lam_in ? sd.lam[0] : sd.lam[1];
    const char *h = reinterpret_cast<const char *>(sd.hist);
    const float *hist1 = reinterpret_cast<const float *>(h + (uint64_t)hist_slot * sd.hist_bytes);
    const float *hist0 =
        reinterpret_cast<const float *>(h + (uint64_t)(hist_slot - 1) * sd.hist_bytes);
    adjoint2_strip<BCX, BCY, KN, FC>(mu_in, mu_out, hist1, hist0, sd.med, sd.mlay, sd.seg,
                                     KN ? sd.seg2 : nullptr, sd.g, sd.ph, band, bnd, strip);
}

// op 0: clear the segment and total planes; 1: fold segment into total;
// 2: write the totals to the output planes.  kn: the ln kn0 plane too.
__global__ __launch_bounds__(256) void batch_grad_kernel(const AdjSampleDesc *__restrict__ samples,
                                                         const int *__restrict__ tile_sample,
                                                         int rows, int op, int kn)
{
    AdjSampleDesc sd;
    uint32_t x;
    int y0, y1;
    if (!adj_tile(samples, tile_sample, rows, sd, x, y0, y1))
        return;
    for (int y = y0; y < y1; ++y) {
        const int64_t c = (int64_t)y * sd.g.pitch + x, o = (int64_t)y * sd.g.nx + x;
        for (int p = 0; p < (kn ? 2 : 1); ++p) {
            float *seg = p ? sd.seg2 : sd.seg;
            double *tot = p ? sd.grad2 : sd.grad;
            if (op == 0) {
                seg[c] = 0.0f;
                tot[c] = 0.0;
            } else if (op == 1) {
                tot[c] += (double)seg[c];
                seg[c] = 0.0f;
            } else {
                (p ? sd.out2 : sd.out)[o] = (float)tot[c];
            }
        }
    }
}

template <int BCX, int BCY>
static hipError_t batch_adj_t(const AdjSampleDesc *samples, const int *tile_sample, int ntiles,
                              int tile_x, int rows, int lam_in, int hist_slot, int kn, int fc,
                              hipStream_t st)
{
#define LBK_BADJK(KN, FC)                                                                    \
    hipLaunchKernelGGL((batch_adjoint_kernel<BCX, BCY, KN, FC>), dim3(ntiles), dim3(tile_x), 0, \
                       st, samples, tile_sample, rows, lam_in, hist_slot)
    if (kn && fc)
        LBK_BADJK(true, true);
    else if (kn)
        LBK_BADJK(true, false);
    else if (fc)
        LBK_BADJK(false, true);
    else
        LBK_BADJK(false, false);
#undef LBK_BADJK
    return hipGetLastError();
}

hipError_t launch_batch_adjoint(int bcx, int bcy, const AdjSampleDesc *samples,
                                const int *tile_sample, int ntiles, int tile_x, int rows,
                                int lam_in, int hist_slot, int kn, int fc, hipStream_t st)
{
    if (tile_x < 64 || tile_x > 256 || (tile_x & 63) || rows < 1 || ntiles < 0)
        return hipErrorInvalidValue;
    if (ntiles == 0)
        return hipSuccess;
#define LBK_BADJ(X, Y)                                                                       \
    batch_adj_t<X, Y>(samples, tile_sample, ntiles, tile_x, rows, lam_in, hist_slot, kn, fc, st)
    switch (bcx * 2 + bcy) {
    case 0: return LBK_BADJ(BC_PERIODIC, BC_PERIODIC);
    case 1: return LBK_BADJ(BC_PERIODIC, BC_WALL);
    case 2: return LBK_BADJ(BC_WALL, BC_PERIODIC);
    case 3: return LBK_BADJ(BC_WALL, BC_WALL);
    case 4: return LBK_BADJ(BC_PRESSURE, BC_PERIODIC);
    case 5: return LBK_BADJ(BC_PRESSURE, BC_WALL);
    default: return hipErrorInvalidValue;
    }
#undef LBK_BADJ
}

template <int BCX, int BCY>
static hipError_t batch_adj2_t(const AdjSampleDesc *samples, const int *tile_sample, int ntiles,
                               int band, int lam_in, int hist_slot, int kn, int fc,
                               hipStream_t st)
{
#define LBK_BADJ2K(KN, FC)                                                                   \
    hipLaunchKernelGGL((batch_adjoint2_kernel<BCX, BCY, KN, FC>), dim3(ntiles), dim3(256), 0,  \
                       st, samples, tile_sample, band, lam_in, hist_slot)
    if (kn && fc)
        LBK_BADJ2K(true, true);
    else if (kn)
        LBK_BADJ2K(true, false);
    else if (fc)
        LBK_BADJ2K(false, true);
    else
        LBK_BADJ2K(false, false);
#undef LBK_BADJ2K
    return hipGetLastError();
}

hipError_t launch_batch_adjoint2(int bcx, int bcy, const AdjSampleDesc *samples,
                                 const int *tile_sample, int ntiles, int band, int lam_in,
                                 int hist_slot, int kn, int fc, hipStream_t st)
{
    if (ntiles < 0 || band < 1 || lam_in < 0 || lam_in > 1 || hist_slot < 1)
        return hipErrorInvalidValue;
    if (ntiles == 0)
        return hipSuccess;
#define LBK_BADJ2(X, Y) batch_adj2_t<X, Y>(samples, tile_sample, ntiles, band, lam_in, hist_slot, kn, fc, st)
    switch (bcx * 2 + bcy) {
    case 0: return LBK_BADJ2(BC_PERIODIC, BC_PERIODIC);
    case 1: return LBK_BADJ2(BC_PERIODIC, BC_WALL);
    case 2: return LBK_BADJ2(BC_WALL, BC_PERIODIC);
    case 3: return LBK_BADJ2(BC_WALL, BC_WALL);
    case 4: return LBK_BADJ2(BC_PRESSURE, BC_PERIODIC);
    case 5: return LBK_BADJ2(BC_PRESSURE, BC_WALL);
    default: return hipErrorInvalidValue;
    }
#undef LBK_BADJ2
}

hipError_t launch_batch_grad(const AdjSampleDesc *samples, const int *tile_sample, int ntiles,
                             int tile_x, int rows, int op, int kn, hipStream_t st)
{
    if (tile_x < 64 || tile_x > 256 || (tile_x & 63) || rows < 1 || ntiles < 0 || op < 0 ||
        op > 2)
        return hipErrorInvalidValue;
    if (ntiles == 0)
        return hipSuccess;
    hipLaunchKernelGGL(batch_grad_kernel, dim3(ntiles), dim3(tile_x), 0, st, samples,
                       tile_sample, rows, op, kn);
    return hipGetLastError();
}

} // namespace lbk
