/*
 * lbo.h -- serial FP64 CPU oracle for the generalized lattice Boltzmann model
 * of porous-medium gas flow with Klinkenberg's effect (Chen, Fang, Kang,
 * Hyman, Viswanathan, Tao; arXiv:1411.7051).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load or call this library.  The product
 * (the HIP path behind include/lbk.h) never links, loads or calls it, and it
 * shares no source with that path.
 *
 * What it computes: the paper's time stepping, written out as plainly as
 * possible, in IEEE double precision, raw (unshifted) populations, two full
 * arrays, one node at a time, phases kept apart (stream, boundary override,
 * collide) exactly in the order the method states them:
 *   - D2Q9 velocities and weights        Eq. 13 and the text after Eq. 14
 *   - BGK evolution                      Eq. 12
 *   - porous equilibrium                 Eq. 14
 *   - Guo forcing term                   Eq. 15 (last term divided by eps, as
 *                                        in Guo's scheme; the printed form is
 *                                        kept behind eq15_printed for tests)
 *   - moments and explicit velocity      Eqs. 16a, 16b, 17 (quadratic root of
 *                                        Eq. 16b when the Forchheimer term of
 *                                        Eq. 2 is on)
 *   - force                              Eq. 8 (Eq. 2 when f_eps != 0)
 *   - apparent permeability              Eq. 3 with Eqs. 6-7
 *   - local Knudsen number               Eq. 5 with Eq. 10 (lambda ~ 1/p)
 *   - node model                         Sec. III: eps = 1 pore, eps = 0 no flow
 *   - walls, pressure inlet/outlet,      Sec. IV.A and IV.B
 *     periodic sides
 *
 * Conventions: lattice units (dx = dt = 1, c = 1, cs^2 = 1/3); arrays are
 * row-major [ny][nx], x fastest; populations are [9][ny][nx].  k = +inf marks
 * a node with no Darcy drag; eps = 0 marks an impermeable node.
 */
#ifndef LBO_H
#define LBO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { LBO_PERIODIC = 0, LBO_WALL = 1, LBO_PRESSURE = 2 };

typedef struct lbo_params {
    int nx, ny;
    double tau;          /* BGK relaxation time, Eq. 12; nu = (tau - 1/2)/3 */
    double gx, gy;       /* external acceleration G of Eqs. 2 and 8 */
    double f_eps;        /* Forchheimer geometric function of Eq. 2; 0 = Eq. 8 */
    int bc_x, bc_y;      /* LBO_PERIODIC / LBO_WALL / LBO_PRESSURE (x only) */
    double rho_in;       /* density imposed on column x = 0 (pressure BC) */
    double rho_out;      /* density imposed on column x = nx-1 */
    double rho0;         /* initial density for a start from rest */
    double rho_ref;      /* density at which kn0 is quoted */
    int kn_local;        /* 1: Kn = kn0 * rho_ref / rho;  0: Kn = kn0 */
    int init;            /* 0: rest at rho0;  1: rest on a linear rho ramp */
    int eq15_printed;    /* test-only: Eq. 15 exactly as printed */
    int correlation;     /* 0: Eqs. 6-7 (second order); 1: Eqs. 4-5 (first
                            order, f_c = 1 + 4 Kn); 2: none (f_c = 1) */
    double slip_b;       /* slip coefficient b of Eq. 6 (R4: -1), <= 0 */
} lbo_params;

typedef struct lbo_lattice lbo_lattice;

/* Eqs. 6-7 with b = -1: the Beskok-Karniadakis/Civan correction factor. */
double lbo_fc(double kn);

/* The correction factor of the selected correlation (see lbo_params). */
double lbo_fc_with(int correlation, double b, double kn);

/* Eq. 14 for one node; out[9]. */
void lbo_feq(double rho, double ux, double uy, double eps, double out[9]);

/* Eq. 15 for one node; out[9]. */
void lbo_guo(double rho, double ux, double uy, double fx, double fy,
             double eps, double tau, int printed, double out[9]);

/* Eqs. 16-17 (+ Eqs. 3, 5-7, 10, 8) for one node from its post-stream
 * populations f[9]: density, velocity and total force. */
void lbo_node_macro(const lbo_params *p, const double f[9], double eps,
                    double k, double kn0, double *rho, double *ux,
                    double *uy, double *fx, double *fy);

/* One collision (Eq. 12 right-hand side) of one node: f_out = f* . */
void lbo_collide_node(const lbo_params *p, const double f[9], double eps,
                      double k, double kn0, double f_out[9]);

/* Create from per-node fields eps, k, kn0 ([ny][nx]; kn0 may be NULL = 0).
 * Returns NULL on invalid input or allocation failure. */
lbo_lattice *lbo_create(const lbo_params *p, const double *eps,
                        const double *k, const double *kn0);
void lbo_destroy(lbo_lattice *L);

/* Advance n time steps. */
void lbo_step(lbo_lattice *L, long n);

/* Macroscopic read-out at the current time: pull-stream, boundary override
 * and Eqs. 16-17 on every node.  Any output pointer may be NULL. */
void lbo_macro(const lbo_lattice *L, double *rho, double *ux, double *uy);

/* Total mass: sum of all post-collision populations. */
double lbo_mass(const lbo_lattice *L);

/* Global (apparent) permeability of the whole domain by Darcy's law. */
double lbo_apparent_permeability(const lbo_lattice *L);

/* Steady-state residual ||u - u_prev||_2 / ||u||_2 (FP64) between two
 * velocity read-outs of n values each (components stacked; the same
 * function serves the D3Q19 oracle); 0 when both are zero, +inf when only
 * u_prev is non-zero. */
double lbo_residual(const double *u, const double *u_prev, size_t n);

/* Post-collision populations f*[9][ny][nx] (copy out / copy in). */
void lbo_get_state(const lbo_lattice *L, double *f);
void lbo_set_state(lbo_lattice *L, const double *f);

/* 1 if any stored population is NaN or infinite. */
int lbo_nonfinite(const lbo_lattice *L);

#ifdef __cplusplus
}
#endif
#endif
