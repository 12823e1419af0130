/*
 * lbo3.c -- D3Q19 form of the FP64 oracle (see lbo3.h).  TEST INFRASTRUCTURE
 * ONLY.  Same structure and readings as lbo.c: raw populations, two arrays,
 * one node at a time, stream -> pressure planes -> collide.
 */
#include "lbo3.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* D3Q19: rest; +-x, +-y, +-z; the twelve face diagonals (pairs with
 * opposite neighbours adjacent). */
static const int EX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int EY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int EZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

static int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

static double weight(int i)
{
    int s = EX[i] * EX[i] + EY[i] * EY[i] + EZ[i] * EZ[i];
    return s == 0 ? 1.0 / 3.0 : (s == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

struct lbo3_lattice {
    lbo3_params p;
    double *eps, *k, *kn0;
    double *f, *fs, *fn; /* [19][nz][ny][nx] */
};

static size_t cell(const lbo3_params *p, int z, int y, int x)
{
    return ((size_t)z * p->ny + y) * p->nx + x;
}

static size_t at(const lbo3_params *p, int i, int z, int y, int x)
{
    return (size_t)i * p->nx * p->ny * p->nz + cell(p, z, y, x);
}

void lbo3_tables(int ex[19], int ey[19], int ez[19], double w[19])
{
    for (int i = 0; i < 19; ++i) {
        ex[i] = EX[i];
        ey[i] = EY[i];
        ez[i] = EZ[i];
        w[i] = weight(i);
    }
}

/* Eq. 14, c = 1. */
void lbo3_feq(double rho, const double u[3], double eps, double out[19])
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < 19; ++i) {
        if (eps == 0.0) { /* R7 */
            out[i] = weight(i) * rho;
            continue;
        }
        double eu = EX[i] * u[0] + EY[i] * u[1] + EZ[i] * u[2];
        out[i] = weight(i) * rho *
                 (1.0 + 3.0 * eu + 9.0 / (2.0 * eps) * eu * eu - 3.0 / (2.0 * eps) * uu);
    }
}

/* Eq. 15, c = 1, with the 1/eps of R1 on the last term. */
void lbo3_guo(double rho, const double u[3], const double F[3], double eps, double tau,
              double out[19])
{
    double c = 1.0 - 1.0 / (2.0 * tau);
    double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    for (int i = 0; i < 19; ++i) {
        double eF = EX[i] * F[0] + EY[i] * F[1] + EZ[i] * F[2];
        double eu = EX[i] * u[0] + EY[i] * u[1] + EZ[i] * u[2];
        double t = 3.0 * eF;
        if (eps > 0.0)
            t += 9.0 / eps * eu * eF - 3.0 / eps * uF;
        out[i] = weight(i) * rho * c * t;
    }
}

/* Eqs. 16-17 with Eqs. 3, 5-7, 8 (2) for one node (the same steps as
 * lbo_node_macro, with three components). */
static void node_macro(const lbo3_params *p, const double f[19], double eps, double k,
                       double kn0, double *rho_out, double u[3], double F[3])
{
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 19; ++i) {
        rho += f[i];
        j[0] += EX[i] * f[i];
        j[1] += EY[i] * f[i];
        j[2] += EZ[i] * f[i];
    }
    const double G[3] = {p->gx, p->gy, p->gz};
    if (eps == 0.0) { /* R7 */
        for (int a = 0; a < 3; ++a) {
            u[a] = 0.0;
            F[a] = -2.0 * j[a] / rho;
        }
    } else {
        double nu = (p->tau - 0.5) / 3.0;
        double kn = p->kn_local ? kn0 * p->rho_ref / rho : kn0;
        double ka = k * lbo_fc_with(p->correlation, p->slip_b, kn); /* Eq. 3 */
        double A = isinf(ka) ? 0.0 : eps * nu / ka;
        double B = (isinf(ka) || p->f_eps == 0.0) ? 0.0 : eps * p->f_eps / sqrt(ka);
        double w[3], wn = 0.0;
        for (int a = 0; a < 3; ++a) {
            w[a] = (j[a] + 0.5 * rho * eps * G[a]) / rho;
            wn += w[a] * w[a];
        }
        wn = sqrt(wn);
        double c0 = 1.0 + 0.5 * A;
        /* Eq. 17, or the rationalized root of Eq. 16b with Eq. 2 (R6) */
        double g = B == 0.0 ? 1.0 / c0 : 2.0 / (c0 + sqrt(c0 * c0 + 2.0 * B * wn));
        double un = 0.0;
        for (int a = 0; a < 3; ++a) {
            u[a] = g * w[a];
            un += u[a] * u[a];
        }
        un = sqrt(un);
        for (int a = 0; a < 3; ++a)
            F[a] = -A * u[a] - B * un * u[a] + eps * G[a]; /* Eq. 2 / Eq. 8 */
    }
    *rho_out = rho;
}

static void collide_node(const lbo3_params *p, const double f[19], double eps, double k,
                         double kn0, double out[19])
{
    double rho, u[3], F[3], feq[19], Fi[19];
    node_macro(p, f, eps, k, kn0, &rho, u, F);
    lbo3_feq(rho, u, eps, feq);
    lbo3_guo(rho, u, F, eps, p->tau, Fi);
    for (int i = 0; i < 19; ++i)
        out[i] = f[i] - (f[i] - feq[i]) / p->tau + Fi[i];
}

/* Pull (Eq. 12 left side) with wrap or bounce-back per axis (R8); links
 * entering a pressure plane from outside are overridden afterwards. */
static void stream(const lbo3_lattice *L)
{
    const lbo3_params *p = &L->p;
    const int bc[3] = {p->bc_x, p->bc_y, p->bc_z}, n[3] = {p->nx, p->ny, p->nz};
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x)
                for (int i = 0; i < 19; ++i) {
                    int s[3] = {x - EX[i], y - EY[i], z - EZ[i]};
                    const int c[3] = {x, y, z};
                    int bounce = 0;
                    for (int a = 0; a < 3; ++a) {
                        if (s[a] >= 0 && s[a] < n[a])
                            continue;
                        if (bc[a] == LBO_WALL)
                            bounce = 1;
                        else if (bc[a] == LBO_PERIODIC)
                            s[a] = (s[a] + n[a]) % n[a];
                        else
                            s[a] = c[a]; /* pressure plane: replaced below */
                    }
                    L->fs[at(p, i, z, y, x)] = bounce ? L->f[at(p, opp(i), z, y, x)]
                                                      : L->f[at(p, i, s[2], s[1], s[0])];
                }
}

/* R9 on the plane x = xb from the neighbouring plane x = xn. */
static void pressure_plane(const lbo3_lattice *L, int xb, int xn, double rho_b)
{
    const lbo3_params *p = &L->p;
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y) {
            size_t cb = cell(p, z, y, xb), cn = cell(p, z, y, xn);
            double fn_[19], eqb[19], eqn[19], rho_n, u[3], F[3];
            for (int i = 0; i < 19; ++i)
                fn_[i] = L->fs[at(p, i, z, y, xn)];
            node_macro(p, fn_, L->eps[cn], L->k[cn], L->kn0[cn], &rho_n, u, F);
            lbo3_feq(rho_b, u, L->eps[cb], eqb);
            lbo3_feq(rho_n, u, L->eps[cn], eqn);
            for (int i = 0; i < 19; ++i)
                L->fs[at(p, i, z, y, xb)] = eqb[i] + fn_[i] - eqn[i];
        }
}

static void stream_and_bound(const lbo3_lattice *L)
{
    stream(L);
    if (L->p.bc_x == LBO_PRESSURE) {
        pressure_plane(L, 0, 1, L->p.rho_in);
        pressure_plane(L, L->p.nx - 1, L->p.nx - 2, L->p.rho_out);
    }
}

lbo3_lattice *lbo3_create(const lbo3_params *p, const double *eps, const double *k,
                          const double *kn0)
{
    if (!p || !eps || !k || p->nx < 1 || p->ny < 1 || p->nz < 1 || !(p->tau > 0.5))
        return NULL;
    if (p->bc_x < 0 || p->bc_x > 2 || p->bc_y < 0 || p->bc_y > 1 || p->bc_z < 0 ||
        p->bc_z > 1)
        return NULL;
    if ((p->bc_x == LBO_PRESSURE || p->init == 1) &&
        (!(p->rho_in > 0.0) || !(p->rho_out > 0.0)))
        return NULL;
    if (p->bc_x == LBO_PRESSURE && p->nx < 3)
        return NULL;
    if (p->init == 0 && !(p->rho0 > 0.0))
        return NULL;
    if (p->correlation < 0 || p->correlation > 2 || !(p->slip_b <= 0.0) || !isfinite(p->slip_b))
        return NULL;
    size_t n = (size_t)p->nx * p->ny * p->nz;
    for (size_t j = 0; j < n; ++j)
        if (!(eps[j] >= 0.0 && eps[j] <= 1.0) || !(k[j] > 0.0) ||
            (kn0 && !(kn0[j] >= 0.0 && isfinite(kn0[j]))))
            return NULL;
    lbo3_lattice *L = (lbo3_lattice *)calloc(1, sizeof *L);
    if (!L)
        return NULL;
    L->p = *p;
    L->eps = (double *)malloc(n * sizeof(double));
    L->k = (double *)malloc(n * sizeof(double));
    L->kn0 = (double *)calloc(n, sizeof(double));
    L->f = (double *)malloc(19 * n * sizeof(double));
    L->fs = (double *)malloc(19 * n * sizeof(double));
    L->fn = (double *)malloc(19 * n * sizeof(double));
    if (!L->eps || !L->k || !L->kn0 || !L->f || !L->fs || !L->fn) {
        lbo3_destroy(L);
        return NULL;
    }
    memcpy(L->eps, eps, n * sizeof(double));
    memcpy(L->k, k, n * sizeof(double));
    if (kn0)
        memcpy(L->kn0, kn0, n * sizeof(double));
    for (int z = 0; z < p->nz; ++z) /* R10 */
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                double rho = p->rho0;
                if (p->init == 1)
                    rho = p->nx > 1 ? p->rho_in + (p->rho_out - p->rho_in) * (double)x /
                                                      (double)(p->nx - 1)
                                    : p->rho_in;
                for (int i = 0; i < 19; ++i)
                    L->f[at(p, i, z, y, x)] = weight(i) * rho;
            }
    return L;
}

void lbo3_destroy(lbo3_lattice *L)
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

void lbo3_step(lbo3_lattice *L, long nsteps)
{
    const lbo3_params *p = &L->p;
    for (long t = 0; t < nsteps; ++t) {
        stream_and_bound(L);
        for (int z = 0; z < p->nz; ++z)
            for (int y = 0; y < p->ny; ++y)
                for (int x = 0; x < p->nx; ++x) {
                    size_t c = cell(p, z, y, x);
                    double f[19], fo[19];
                    for (int i = 0; i < 19; ++i)
                        f[i] = L->fs[at(p, i, z, y, x)];
                    collide_node(p, f, L->eps[c], L->k[c], L->kn0[c], fo);
                    for (int i = 0; i < 19; ++i)
                        L->fn[at(p, i, z, y, x)] = fo[i];
                }
        double *tmp = L->f;
        L->f = L->fn;
        L->fn = tmp;
    }
}

void lbo3_macro(const lbo3_lattice *L, double *rho, double *ux, double *uy, double *uz)
{
    const lbo3_params *p = &L->p;
    stream_and_bound(L);
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                size_t c = cell(p, z, y, x);
                double f[19], r, u[3], F[3];
                for (int i = 0; i < 19; ++i)
                    f[i] = L->fs[at(p, i, z, y, x)];
                node_macro(p, f, L->eps[c], L->k[c], L->kn0[c], &r, u, F);
                if (rho)
                    rho[c] = r;
                if (ux)
                    ux[c] = u[0];
                if (uy)
                    uy[c] = u[1];
                if (uz)
                    uz[c] = u[2];
            }
}

double lbo3_mass(const lbo3_lattice *L)
{
    size_t n = 19 * (size_t)L->p.nx * L->p.ny * L->p.nz;
    double m = 0.0;
    for (size_t j = 0; j < n; ++j)
        m += L->f[j];
    return m;
}

/* R11 with the mean over every node and eps_b over the two pressure planes. */
double lbo3_apparent_permeability(const lbo3_lattice *L)
{
    const lbo3_params *p = &L->p;
    size_t n = (size_t)p->nx * p->ny * p->nz;
    double *rho = (double *)malloc(n * sizeof(double));
    double *ux = (double *)malloc(n * sizeof(double));
    if (!rho || !ux) {
        free(rho);
        free(ux);
        return NAN;
    }
    lbo3_macro(L, rho, ux, NULL, NULL);
    double q = 0.0, u = 0.0;
    for (size_t j = 0; j < n; ++j) {
        q += rho[j] * ux[j];
        u += ux[j];
    }
    q /= (double)n;
    u /= (double)n;
    free(rho);
    free(ux);
    double nu = (p->tau - 0.5) / 3.0;
    if (p->bc_x == LBO_PRESSURE) {
        double eb = 0.0;
        for (int z = 0; z < p->nz; ++z)
            for (int y = 0; y < p->ny; ++y)
                eb += L->eps[cell(p, z, y, 0)] + L->eps[cell(p, z, y, p->nx - 1)];
        eb /= 2.0 * p->ny * p->nz;
        return eb * nu * (double)(p->nx - 1) * q / ((1.0 / 3.0) * (p->rho_in - p->rho_out));
    }
    return nu * u / p->gx;
}

void lbo3_get_state(const lbo3_lattice *L, double *f)
{
    memcpy(f, L->f, 19 * (size_t)L->p.nx * L->p.ny * L->p.nz * sizeof(double));
}

void lbo3_set_state(lbo3_lattice *L, const double *f)
{
    memcpy(L->f, f, 19 * (size_t)L->p.nx * L->p.ny * L->p.nz * sizeof(double));
}
