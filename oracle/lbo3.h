/*
 * lbo3.h -- serial FP64 CPU oracle of the same Klinkenberg lattice Boltzmann
 * model (arXiv:1411.7051) on a three-dimensional D3Q19 lattice.
 *
 * TEST INFRASTRUCTURE ONLY, like lbo.h: only tests/, the smoke check and the
 * benchmark's CPU baseline may load it; the product never links or calls it.
 *
 * The paper's model (Eqs. 12, 14-17 with Eqs. 2-8) is written for any
 * lattice; this is its D3Q19 form: nineteen velocities (rest, six axis
 * links, twelve face diagonals) with weights 1/3, 1/18 and 1/36, cs^2 = 1/3.
 * The equilibrium of Eq. 14 and Guo's forcing of Eq. 15 keep their form with
 * three-component vectors; Eqs. 16-17 and the force of Eq. 8 (Eq. 2) are
 * unchanged.  Readings R1-R11 of lbo.h apply as stated there, with the
 * pressure boundary imposed on the planes x = 0 and x = nx-1 and walls
 * possible in x, y and z.
 */
#ifndef LBO3_H
#define LBO3_H

#include "lbo.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbo3_params {
    int nx, ny, nz;
    double tau;
    double gx, gy, gz;   /* external acceleration G */
    double f_eps;        /* Forchheimer function of Eq. 2; 0 = Eq. 8 */
    int bc_x, bc_y, bc_z; /* LBO_PERIODIC / LBO_WALL; LBO_PRESSURE in x only */
    double rho_in, rho_out, rho0, rho_ref;
    int kn_local, init, correlation;
    double slip_b;
} lbo3_params;

typedef struct lbo3_lattice lbo3_lattice;

/* The D3Q19 velocity set and weights as used here (for tests). */
void lbo3_tables(int ex[19], int ey[19], int ez[19], double w[19]);

/* Eq. 14 in three dimensions for one node; out[19]. */
void lbo3_feq(double rho, const double u[3], double eps, double out[19]);

/* Eq. 15 (R1) in three dimensions for one node; out[19]. */
void lbo3_guo(double rho, const double u[3], const double F[3], double eps, double tau,
              double out[19]);

/* Fields eps, k, kn0 are [nz][ny][nx] (kn0 may be NULL); NULL on invalid
 * input. */
lbo3_lattice *lbo3_create(const lbo3_params *p, const double *eps, const double *k,
                          const double *kn0);
void lbo3_destroy(lbo3_lattice *L);
void lbo3_step(lbo3_lattice *L, long n);

/* Read-out (Eqs. 16-17 on the post-stream populations); NULLs allowed. */
void lbo3_macro(const lbo3_lattice *L, double *rho, double *ux, double *uy, double *uz);
double lbo3_mass(const lbo3_lattice *L);
double lbo3_apparent_permeability(const lbo3_lattice *L);
/* Post-collision populations [19][nz][ny][nx]. */
void lbo3_get_state(const lbo3_lattice *L, double *f);
void lbo3_set_state(lbo3_lattice *L, const double *f);

#ifdef __cplusplus
}
#endif
#endif
