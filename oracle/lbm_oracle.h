/*
 * lbm_oracle.h -- CPU reference ("oracle") for the rectangular-lattice
 * central-moment LBM of Yahia & Premnath (arXiv 2103.02119).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU-baseline leg of the benchmark can compare the HIP
 * library against a plain, slow, obviously correct implementation.  The
 * product path never links, loads or calls it.  It shares no code, header,
 * table or constant generator with the HIP library.
 *
 * Everything is FP64 and written from the definitions: raw moments as sums
 * of the basis monomials of Eq. 3 over the populations, central moments as
 * the same sums about the node's velocity (Eq. 43), and the way back to
 * populations as the solution of the 9 x 9 linear system "these
 * populations have these moments" (Gaussian elimination); raw equilibria
 * (Eq. 12), raw sources (Eq. 13), central equilibria (Eq. 49), corrections
 * (Eq. 23-27), local strain rate (Eq. 37-38, coefficients Eq. 40), RNR
 * collision (Sec. 3), RC collision (Sec. 4), perfect-shift streaming,
 * half-way bounce-back and the moving-wall correction (Sec. 5.2,
 * Eq. 57-59).  The matrices the paper prints (T of Eq. 4, T^{-1} of App. A,
 * F(u) of Eq. 53) are exported for the tests that pin them; the scheme
 * does not use T^{-1} or F.
 *
 * Layout of every field: [9][ny][nx] for populations, [ny][nx] for scalar
 * fields, x fastest.  Node (i, j) sits at x = i (+1/2), y = (j + 1/2) * a.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_RC = 0, ORC_RNR = 1 };
enum { ORC_PERIODIC = 0, ORC_WALL = 1, ORC_MOVING_WALL = 2 };
/* face index: 0 = x-min, 1 = x-max, 2 = y-min, 3 = y-max */

typedef struct {
    int nx, ny;
    double a;          /* grid aspect ratio dy/dx (Sec. 2.1) */
    double cs2;        /* squared speed of sound */
    double rho0;       /* reference density; also the wall density rho_w */
    double omega[9];   /* relaxation rates omega_0..omega_8 */
    double force[2];   /* uniform body force (Fx, Fy) */
    int collision;     /* ORC_RC or ORC_RNR */
    int corrections;   /* 1: add Eq. 23-26 corrections; 0: leave them out */
    int bc_type[4];    /* per face, ORC_PERIODIC / ORC_WALL / ORC_MOVING_WALL */
    double u_wall[4][2];
    /* optional obstacle mask [ny][nx], nonzero = solid node (NULL: none).
     * A link whose source node is solid bounces back half-way at rest
     * (Sec. 5.2 with u_w = 0); a solid neighbour's density is replaced by the
     * node's own in the density gradient (as at a wall); solid nodes hold the
     * rest state feq(rho0, 0). */
    const unsigned char *solid;
} orc_params;

/* --- matrices (row-major 9x9) --- */
void orc_T(double a, double *T);
void orc_Tinv(double a, double *Ti);
void orc_F(double ux, double uy, double *F);

/* --- per-node pieces --- */
void orc_macro(const orc_params *p, const double *f9, double *rho, double *ux, double *uy);
void orc_feq(const orc_params *p, double rho, double ux, double uy, double *feq9);
void orc_strain_rate(const orc_params *p, const double *f9, double drho_dx, double drho_dy,
                     double *dux_dx, double *duy_dy);
void orc_corrections(const orc_params *p, const double *f9, double drho_dx, double drho_dy,
                     double *delta3, double *delta4);
void orc_collide_node(const orc_params *p, const double *f9, double drho_dx, double drho_dy,
                      double *out9);

/* --- whole-field operations --- */
void orc_init(const orc_params *p, const double *rho, const double *ux, const double *uy,
              double *f);
void orc_density(const orc_params *p, const double *f, double *rho);
void orc_density_gradient(const orc_params *p, const double *rho, double *gx, double *gy);
void orc_collide(const orc_params *p, const double *f, double *ft);
void orc_stream(const orc_params *p, const double *ft, double *f);
void orc_step_node(const orc_params *p, const double *f, int i, int j, double *out9);
void orc_run(const orc_params *p, double *f, double *work, long nsteps);
void orc_moments(const orc_params *p, const double *f, double *rho, double *ux, double *uy);
void orc_stress(const orc_params *p, const double *f, double *sxx, double *syy, double *sxy);

int orc_max_threads(void);
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
