/*
 * lbo.c -- serial FP64 CPU oracle for the Klinkenberg lattice Boltzmann model
 * of arXiv:1411.7051.  TEST INFRASTRUCTURE ONLY (see lbo.h): the product path
 * never loads, links or calls it.
 *
 * Written for a reader holding the paper: every function names the equation
 * or passage it follows, works in IEEE double precision on raw populations,
 * and keeps the method's phases apart (stream, boundary override, moments,
 * collide).  Built with -O2 -ffp-contract=off and no fast-math.
 *
 * Readings where the paper is silent or garbled (each is also listed with
 * its reason in the design notes of the repository):
 *   R1  Eq. 15's last term carries 1/eps, as in Guo's forcing scheme that
 *       Sec. III adopts; the printed term without it does not conserve mass.
 *       The printed form stays reachable through eq15_printed (tests only).
 *   R2  nu = nu_e = (tau - 1/2)/3 in lattice units, viscosity ratio J = 1
 *       (Sec. IV.A), c = 1, cs^2 = 1/3.
 *   R3  Kn = 0 gives f_c = 1 exactly (Eq. 7 is singular there; Sec. III says
 *       the model then reduces to Guo's).
 *   R4  b = -1 in Eq. 6 for every regime.
 *   R5  Kn is local: Kn = kn0 * rho_ref / rho, since Eq. 10 gives
 *       lambda ~ 1/p at fixed temperature and viscosity (Eq. 5: Kn = lambda/r).
 *   R6  With the Forchheimer term of Eq. 2 on, Eq. 16b is quadratic in |u|;
 *       its positive root is taken in rationalized form.
 *   R7  Impermeable node (eps = 0): Sec. III gives it infinite drag and zero
 *       velocity.  Eq. 17 with the Darcy coefficient of Eq. 8 going to
 *       infinity gives u -> 0 while the force tends to the finite value that
 *       Eq. 16b needs for u = 0, rho F = -2 sum_i f_i e_i; the terms of
 *       Eqs. 14-15 that divide by eps carry u and vanish in that limit, so
 *       f_eq = w_i rho and F_i = w_i rho (1 - 1/2tau) 3 e_i.F.
 *   R8  Walls: half-way bounce-back (walls half a link outside the first and
 *       last rows or columns).
 *   R9  Pressure inlet/outlet: non-equilibrium extrapolation from the
 *       neighbouring column on all nine post-stream populations.
 *   R10 Start from rest: f = w_i rho0, or w_i rho(x) on a linear density
 *       ramp between rho_in and rho_out.
 *   R11 Global permeability: Darcy's law over the whole domain (Sec. IV.A),
 *       see lbo_apparent_permeability.
 *   R13 Steady state (Sec. IV.A) is measured by the relative L2 change of
 *       the velocity field between two read-outs, see lbo_residual.
 */
#include "lbo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Eq. 13.  i = 0: rest; i = 1..4: unit vectors at angles (i-1)*pi/2;
 * i = 5..8: sqrt(2) * unit vectors at angles (i-5)*pi/2 + pi/4. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* Direction opposite to i: e_OPP[i] = -e_i. */
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
/* Weights stated after Eq. 14: 4/9, 1/9 (axis), 1/36 (diagonal). */
static const double W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                            1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

struct lbo_lattice {
    lbo_params p;
    double *eps, *k, *kn0; /* per-node medium, [ny][nx] */
    double *f;             /* post-collision populations f*, [9][ny][nx] */
    double *fs;            /* post-stream populations (scratch) */
    double *fn;            /* next post-collision populations (scratch) */
};

static size_t at(const lbo_params *p, int i, int y, int x)
{
    return ((size_t)i * (size_t)p->ny + (size_t)y) * (size_t)p->nx + (size_t)x;
}

static double viscosity(const lbo_params *p)
{
    return (p->tau - 0.5) / 3.0; /* R2 */
}

/* Eqs. 6-7: f_c = (1 + alpha Kn) [1 + 4 Kn / (1 - b Kn)], b = -1,
 * alpha = 1.358 / (1 + 0.170 Kn^-0.4348). */
double lbo_fc_with(int correlation, double b, double kn)
{
    if (!(kn > 0.0) || correlation == 2)
        return 1.0; /* R3; or no slip correction */
    if (correlation == 1)
        return 1.0 + 4.0 * kn; /* Eqs. 4-5, c = 1 */
    double alpha = 1.358 / (1.0 + 0.170 * pow(kn, -0.4348)); /* Eq. 7 */
    return (1.0 + alpha * kn) * (1.0 + 4.0 * kn / (1.0 - b * kn)); /* Eq. 6 */
}

double lbo_fc(double kn) { return lbo_fc_with(0, -1.0 /* R4 */, kn); }

/* Eq. 14 with c = 1. */
void lbo_feq(double rho, double ux, double uy, double eps, double out[9])
{
    for (int i = 0; i < 9; ++i) {
        if (eps == 0.0) { /* R7: u = 0 at an impermeable node */
            out[i] = W[i] * rho;
            continue;
        }
        double eu = EX[i] * ux + EY[i] * uy;
        double uu = ux * ux + uy * uy;
        out[i] = W[i] * rho *
                 (1.0 + 3.0 * eu + 9.0 / (2.0 * eps) * eu * eu -
                  3.0 / (2.0 * eps) * uu);
    }
}

/* Eq. 15 with c = 1, dt = 1 (R1 for the last term). */
void lbo_guo(double rho, double ux, double uy, double fx, double fy,
             double eps, double tau, int printed, double out[9])
{
    for (int i = 0; i < 9; ++i) {
        double eF = EX[i] * fx + EY[i] * fy;
        if (eps == 0.0) { /* R7: u = 0, the 1/eps terms vanish */
            out[i] = W[i] * rho * (1.0 - 1.0 / (2.0 * tau)) * 3.0 * eF;
            continue;
        }
        double eu = EX[i] * ux + EY[i] * uy;
        double uF = ux * fx + uy * fy;
        double last = printed ? 3.0 * uF : 3.0 / eps * uF;
        out[i] = W[i] * rho * (1.0 - 1.0 / (2.0 * tau)) *
                 (3.0 * eF + 9.0 / eps * eu * eF - last);
    }
}

/* Eq. 16a, Eq. 16b solved through Eq. 17 (or its quadratic, R6), with the
 * apparent permeability of Eq. 3 / Eqs. 6-7 at the local Kn (R5) and the
 * force of Eq. 8 (Eq. 2 when f_eps != 0). */
void lbo_node_macro(const lbo_params *p, const double f[9], double eps,
                    double k, double kn0, double *rho_out, double *ux_out,
                    double *uy_out, double *fx_out, double *fy_out)
{
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < 9; ++i) {
        rho += f[i];
        jx += EX[i] * f[i];
        jy += EY[i] * f[i];
    }
    double ux = 0.0, uy = 0.0, fx, fy;
    if (eps == 0.0) {
        /* R7: infinite drag; Eq. 16b with u = 0 fixes rho F = -2 j */
        fx = -2.0 * jx / rho;
        fy = -2.0 * jy / rho;
    } else {
        double nu = viscosity(p);
        double kn = p->kn_local ? kn0 * p->rho_ref / rho : kn0;
        double ka = k * lbo_fc_with(p->correlation, p->slip_b, kn); /* Eq. 3 */
        double A = isinf(ka) ? 0.0 : eps * nu / ka;      /* Darcy, Eq. 8 */
        double B = (isinf(ka) || p->f_eps == 0.0)
                       ? 0.0
                       : eps * p->f_eps / sqrt(ka);      /* Forchheimer, Eq. 2 */
        double vx = jx + 0.5 * rho * eps * p->gx;
        double vy = jy + 0.5 * rho * eps * p->gy;
        if (B == 0.0) {
            /* Eq. 17 */
            double den = rho + 0.5 * A * rho;
            ux = vx / den;
            uy = vy / den;
        } else {
            /* Eq. 16b with Eq. 2:  (1 + A/2) u + (B/2)|u| u = v / rho, so u
             * is parallel to w = v / rho and |u| is the positive root of
             * (B/2) s^2 + (1 + A/2) s - |w| = 0, written rationalized:
             * s = 2|w| / (c0 + sqrt(c0^2 + 2 B |w|)). */
            double wx = vx / rho, wy = vy / rho;
            double wn = sqrt(wx * wx + wy * wy);
            double c0 = 1.0 + 0.5 * A;
            double g = 2.0 / (c0 + sqrt(c0 * c0 + 2.0 * B * wn));
            ux = g * wx;
            uy = g * wy;
        }
        double un = sqrt(ux * ux + uy * uy);
        fx = -A * ux - B * un * ux + eps * p->gx;
        fy = -A * uy - B * un * uy + eps * p->gy;
    }
    *rho_out = rho;
    *ux_out = ux;
    *uy_out = uy;
    *fx_out = fx;
    *fy_out = fy;
}

/* Right-hand side of Eq. 12 for one node (dt = 1). */
void lbo_collide_node(const lbo_params *p, const double f[9], double eps,
                      double k, double kn0, double f_out[9])
{
    double rho, ux, uy, fx, fy, feq[9], F[9];
    lbo_node_macro(p, f, eps, k, kn0, &rho, &ux, &uy, &fx, &fy);
    lbo_feq(rho, ux, uy, eps, feq);
    lbo_guo(rho, ux, uy, fx, fy, eps, p->tau, p->eq15_printed, F);
    for (int i = 0; i < 9; ++i)
        f_out[i] = f[i] - (f[i] - feq[i]) / p->tau + F[i];
}

/* Left-hand side of Eq. 12 as a pull: f_i(x) = f*_i(x - e_i).  A link that
 * crosses a wall returns the opposite population of the same node (R8);
 * periodic axes wrap; links entering a pressure column from outside are
 * left as placeholders (the whole column is overridden afterwards). */
static void stream(const lbo_lattice *L, const double *src, double *dst)
{
    const lbo_params *p = &L->p;
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x)
            for (int i = 0; i < 9; ++i) {
                int xs = x - EX[i], ys = y - EY[i];
                int bounce = 0;
                if (ys < 0 || ys >= p->ny) {
                    if (p->bc_y == LBO_WALL)
                        bounce = 1;
                    else
                        ys = (ys + p->ny) % p->ny;
                }
                if (xs < 0 || xs >= p->nx) {
                    if (p->bc_x == LBO_WALL)
                        bounce = 1;
                    else if (p->bc_x == LBO_PERIODIC)
                        xs = (xs + p->nx) % p->nx;
                    else
                        xs = x; /* pressure column: replaced below */
                }
                dst[at(p, i, y, x)] = bounce ? src[at(p, OPP[i], y, x)]
                                             : src[at(p, i, ys, xs)];
            }
}

/* R9: on column xb, with neighbour column xn, impose density rho_b:
 * f_i(xb) = f_eq_i(rho_b, u_n; eps_b) + f_i(xn) - f_eq_i(rho_n, u_n; eps_n). */
static void pressure_column(const lbo_lattice *L, double *fs, int xb, int xn,
                            double rho_b)
{
    const lbo_params *p = &L->p;
    for (int y = 0; y < p->ny; ++y) {
        size_t nb = (size_t)y * p->nx + xb, nn = (size_t)y * p->nx + xn;
        double fn_[9], eqb[9], eqn[9];
        for (int i = 0; i < 9; ++i)
            fn_[i] = fs[at(p, i, y, xn)];
        double rho_n, ux, uy, fx, fy;
        lbo_node_macro(p, fn_, L->eps[nn], L->k[nn], L->kn0[nn], &rho_n, &ux,
                       &uy, &fx, &fy);
        lbo_feq(rho_b, ux, uy, L->eps[nb], eqb);
        lbo_feq(rho_n, ux, uy, L->eps[nn], eqn);
        for (int i = 0; i < 9; ++i)
            fs[at(p, i, y, xb)] = eqb[i] + fn_[i] - eqn[i];
    }
}

/* Stream the current state into L->fs and apply the boundary override. */
static void stream_and_bound(const lbo_lattice *L)
{
    const lbo_params *p = &L->p;
    stream(L, L->f, L->fs);
    if (p->bc_x == LBO_PRESSURE) {
        /* both columns read column 1 / nx-2, which are never overridden */
        pressure_column(L, L->fs, 0, 1, p->rho_in);
        pressure_column(L, L->fs, p->nx - 1, p->nx - 2, p->rho_out);
    }
}

lbo_lattice *lbo_create(const lbo_params *p, const double *eps,
                        const double *k, const double *kn0)
{
    if (!p || !eps || !k)
        return NULL;
    if (p->nx < 1 || p->ny < 1 || !(p->tau > 0.5))
        return NULL;
    if (p->bc_x < 0 || p->bc_x > 2 || p->bc_y < 0 || p->bc_y > 1)
        return NULL;
    if (p->bc_x == LBO_PRESSURE &&
        (p->nx < 3 || !(p->rho_in > 0.0) || !(p->rho_out > 0.0)))
        return NULL;
    if (p->init == 0 && !(p->rho0 > 0.0))
        return NULL;
    if (p->correlation < 0 || p->correlation > 2 || !(p->slip_b <= 0.0) || !isfinite(p->slip_b))
        return NULL;
    if (p->init == 1 && (!(p->rho_in > 0.0) || !(p->rho_out > 0.0)))
        return NULL;
    size_t n = (size_t)p->nx * (size_t)p->ny;
    for (size_t j = 0; j < n; ++j) {
        if (!(eps[j] >= 0.0 && eps[j] <= 1.0))
            return NULL;
        if (!(k[j] > 0.0)) /* +inf allowed, NaN rejected */
            return NULL;
        if (kn0 && !(kn0[j] >= 0.0 && isfinite(kn0[j])))
            return NULL;
    }
    lbo_lattice *L = (lbo_lattice *)calloc(1, sizeof *L);
    if (!L)
        return NULL;
    L->p = *p;
    L->eps = (double *)malloc(n * sizeof(double));
    L->k = (double *)malloc(n * sizeof(double));
    L->kn0 = (double *)calloc(n, sizeof(double));
    L->f = (double *)malloc(9 * n * sizeof(double));
    L->fs = (double *)malloc(9 * n * sizeof(double));
    L->fn = (double *)malloc(9 * n * sizeof(double));
    if (!L->eps || !L->k || !L->kn0 || !L->f || !L->fs || !L->fn) {
        lbo_destroy(L);
        return NULL;
    }
    memcpy(L->eps, eps, n * sizeof(double));
    memcpy(L->k, k, n * sizeof(double));
    if (kn0)
        memcpy(L->kn0, kn0, n * sizeof(double));
    /* R10: equilibrium at rest, f_i = w_i rho. */
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            double rho = p->rho0;
            if (p->init == 1)
                rho = p->nx > 1 ? p->rho_in + (p->rho_out - p->rho_in) *
                                                  (double)x / (double)(p->nx - 1)
                                : p->rho_in;
            for (int i = 0; i < 9; ++i)
                L->f[at(p, i, y, x)] = W[i] * rho;
        }
    return L;
}

void lbo_destroy(lbo_lattice *L)
{
    if (!L)
        return;
    free(L->eps);
    free(L->k);
    free(L->kn0);
    free(L->f);
    free(L->fs);
    free(L->fn);
    free(L);
}

/* Eq. 12, n times: stream (+ boundary override), then collide every node. */
void lbo_step(lbo_lattice *L, long n)
{
    const lbo_params *p = &L->p;
    for (long t = 0; t < n; ++t) {
        stream_and_bound(L);
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                size_t c = (size_t)y * p->nx + x;
                double f[9], fo[9];
                for (int i = 0; i < 9; ++i)
                    f[i] = L->fs[at(p, i, y, x)];
                lbo_collide_node(p, f, L->eps[c], L->k[c], L->kn0[c], fo);
                for (int i = 0; i < 9; ++i)
                    L->fn[at(p, i, y, x)] = fo[i];
            }
        double *tmp = L->f;
        L->f = L->fn;
        L->fn = tmp;
    }
}

/* Eqs. 16-17 on the post-stream populations of the current time. */
void lbo_macro(const lbo_lattice *L, double *rho, double *ux, double *uy)
{
    const lbo_params *p = &L->p;
    stream_and_bound(L);
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            size_t c = (size_t)y * p->nx + x;
            double f[9], r, u, v, fx, fy;
            for (int i = 0; i < 9; ++i)
                f[i] = L->fs[at(p, i, y, x)];
            lbo_node_macro(p, f, L->eps[c], L->k[c], L->kn0[c], &r, &u, &v,
                           &fx, &fy);
            if (rho)
                rho[c] = r;
            if (ux)
                ux[c] = u;
            if (uy)
                uy[c] = v;
        }
}

double lbo_mass(const lbo_lattice *L)
{
    size_t n = 9 * (size_t)L->p.nx * (size_t)L->p.ny;
    double m = 0.0;
    for (size_t j = 0; j < n; ++j)
        m += L->f[j];
    return m;
}

/* R11.  Body-force drive: k = nu <u_x> / G_x (Darcy: u = k G / nu).
 * Pressure drive: k = eps_b nu L <rho u_x> / (cs^2 (rho_in - rho_out)) with
 * L = nx - 1 and eps_b the mean porosity of the two pressure columns, since
 * the pressure gradient term of Eq. 1b is grad(eps p) / rho and eps p =
 * cs^2 rho in this model.  <.> is the mean over every node. */
double lbo_apparent_permeability(const lbo_lattice *L)
{
    const lbo_params *p = &L->p;
    size_t n = (size_t)p->nx * (size_t)p->ny;
    double *rho = (double *)malloc(n * sizeof(double));
    double *ux = (double *)malloc(n * sizeof(double));
    if (!rho || !ux) {
        free(rho);
        free(ux);
        return NAN;
    }
    lbo_macro(L, rho, ux, NULL);
    double q = 0.0, u = 0.0;
    for (size_t j = 0; j < n; ++j) {
        q += rho[j] * ux[j];
        u += ux[j];
    }
    q /= (double)n;
    u /= (double)n;
    free(rho);
    free(ux);
    double nu = viscosity(p);
    if (p->bc_x == LBO_PRESSURE) {
        double eb = 0.0;
        for (int y = 0; y < p->ny; ++y)
            eb += L->eps[(size_t)y * p->nx] +
                  L->eps[(size_t)y * p->nx + p->nx - 1];
        eb /= 2.0 * p->ny;
        return eb * nu * (double)(p->nx - 1) * q /
               ((1.0 / 3.0) * (p->rho_in - p->rho_out));
    }
    return nu * u / p->gx;
}

/* Steady-state residual of R13 (Sec. IV.A runs "to steady state" without
 * defining the measure): the relative change of the velocity field between
 * two read-outs, ||u - u_prev||_2 / ||u||_2, in FP64 over the n values of
 * every velocity component of every node (u and u_prev hold the components
 * one after another).  0 when both fields are zero; +inf when u is zero
 * and u_prev is not. */
double lbo_residual(const double *u, const double *u_prev, size_t n)
{
    double dd = 0.0, uu = 0.0;
    for (size_t j = 0; j < n; ++j) {
        double d = u[j] - u_prev[j];
        dd += d * d;
        uu += u[j] * u[j];
    }
    if (uu == 0.0)
        return dd == 0.0 ? 0.0 : INFINITY;
    return sqrt(dd / uu);
}

void lbo_get_state(const lbo_lattice *L, double *f)
{
    memcpy(f, L->f, 9 * (size_t)L->p.nx * (size_t)L->p.ny * sizeof(double));
}

void lbo_set_state(lbo_lattice *L, const double *f)
{
    memcpy(L->f, f, 9 * (size_t)L->p.nx * (size_t)L->p.ny * sizeof(double));
}

int lbo_nonfinite(const lbo_lattice *L)
{
    size_t n = 9 * (size_t)L->p.nx * (size_t)L->p.ny;
    for (size_t j = 0; j < n; ++j)
        if (!isfinite(L->f[j]))
            return 1;
    return 0;
}
