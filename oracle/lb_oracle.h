/*
 * Oracle for the free-energy MRT lattice Boltzmann capillary-filling scheme of
 * Pooley, Kusumaatmaja & Yeomans, "Modelling capillary filling dynamics using
 * lattice Boltzmann simulations" (arXiv:0911.0459).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 CPU implementation
 * written to check the GPU library against.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the product path never
 * does.  It shares no code, header, table or constant with the GPU library.
 *
 * Parity unpinned: which ghost a node at a convex lip of the tube takes in the
 * wall rule of the stencils (through the node; the paper does not say, and no
 * symmetry or closed form fixes it; the flat-wall gradient and the mirror
 * symmetry of the two lips are pinned).  orc_set_wall_gradient only replaces
 * the gradient the following steps use.
 */
#ifndef LB_ORACLE_H
#define LB_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_EUNSTABLE = -4 };
enum { ORC_VDW = 0, ORC_BINARY = 1 };

typedef struct {
    int    model;        /* ORC_VDW or ORC_BINARY */
    double kappa;        /* gradient coefficient (both models) */
    double a, b, T;      /* van der Waals p0 = rho T/(1-b rho) - a rho^2 (Sec. 2) */
    double A, B;         /* phi^4 free energy: mu = -A phi + B phi^3 - kappa lap phi (Sec. 3.1) */
    double Gamma;        /* coefficient 2M/dt of mu in g^eq (Appendix A) */
    double nu_l, nu_g;   /* kinematic viscosities; vdW uses nu_l (Eq. nu for binary) */
    double wall_grad;    /* prescribed normal gradient of rho/phi at the wall, n into fluid */
    double force_x;      /* uniform body force along x (Guo forcing); 0 in capillary runs */
    int    lambda_mode;  /* 0: Chapman-Enskog lambda for vdW (traceless and isotropic
                            parts of the Galilean term each with the rate of its own
                            moment), 1: lambda = 0; 2 and 3: test-only variants (orc_feq) */
} orc_params;

typedef struct {
    int nx, ny;          /* lattice size, x periodic, y periodic where no wall */
    int x_in, tube_len;  /* tube section x in [x_in, x_in+tube_len); tube_len 0 = no tube */
    int tube_h, y0;      /* channel rows [y0, y0+tube_h) are fluid inside the tube section */
} orc_geom;

typedef struct orc_state orc_state;

const char* orc_error(void);
int orc_threads(void);   /* OpenMP threads the oracle's loops use */

/* Build the state at t = 0: f = f^eq, g = g^eq of the initial field init_q
 * (ny*nx, row-major, y major): rho for vdW, phi for binary (rho = 1). */
int  orc_create(const orc_params* p, const orc_geom* g, const double* init_q, orc_state** out);
/* The same with an initial velocity field (ny*nx each, NULL = 0): f = f^eq(q, u). */
int  orc_create_flow(const orc_params* p, const orc_geom* g, const double* init_q,
                     const double* init_ux, const double* init_uy, orc_state** out);
void orc_free(orc_state* s);
int  orc_step(orc_state* s, long nsteps);
long orc_time(const orc_state* s);
/* Change the wall gradient (normal derivative of rho/phi at the wall) for the
 * steps that follow: the equilibrium gradient scanned in time, Sec. 2.2, Fig. 2. */
int  orc_set_wall_gradient(orc_state* s, double wall_grad);

/* Macroscopic fields of the current (post-stream, post-rest) state; solid nodes get 0. */
void orc_moments(const orc_state* s, double* rho, double* ux, double* uy, double* phi);
/* Populations [9][ny][nx]: which = 0 for f, 1 for g. */
void orc_get_pop(const orc_state* s, int which, double* out);
/* Filled length l and l_eff = l + H/2 (Fig. 1b) from the centreline crossing of q_mid. */
int  orc_interface_length(const orc_state* s, double q_mid, double* l, double* l_eff);

/* Pieces exposed for the unit pins. */
void orc_matrix_M(double* out81);
void orc_matrix_Minv(double* out81);
void orc_solid_mask(const orc_geom* g, unsigned char* mask);
int  orc_gradients(const orc_geom* g, double wall_grad, const double* q,
                   double* dxq, double* dyq, double* lapq);
void orc_feq(const orc_params* p, double rho, double ux, double uy, double omega,
             double X, double dxq, double dyq, double* feq);
void orc_geq(const orc_params* p, double phi, double ux, double uy, double mu, double* geq);
void orc_collide(const orc_params* p, const double* f, const double* feq, double omega,
                 double ux, double uy, double Fx, double Fy, double* fstar);

#ifdef __cplusplus
}
#endif
#endif
