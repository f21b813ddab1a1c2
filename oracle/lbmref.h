/*
 * lbmref.h -- plain FP64 CPU oracle for the force-approach pseudopotential
 * lattice Boltzmann update (Czelusniak, Mapelli, Guzella, Cabezas-Gomez,
 * Wagner, "Force approach for the pseudopotential lattice Boltzmann method",
 * arXiv:2003.07968).
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle exists so that tests can check the
 * HIP path against an obviously correct, slow implementation written straight
 * from the paper's equations.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product library never does,
 * and the two share no code, header, table or helper.
 *
 * Conventions (all buffers are caller-owned host memory):
 *   - fields are row-major [ny][nx], x fastest: cell (x, y) is at y*nx + x;
 *   - populations are [9][ny][nx], direction-major, in the order of the D2Q9
 *     velocity set of Sec. II.A (Eq. VelocitySet): i = 0 rest; 1..4 = +x, +y,
 *     -x, -y; 5..8 = (+1,+1), (-1,+1), (-1,-1), (+1,-1);
 *   - the state at time t is the post-streaming, pre-collision f(t); one step
 *     collides (Eq. TLBE right-hand side) and then streams to f(t+1);
 *   - boundaries are periodic in x and y.
 */
#ifndef LBMREF_H
#define LBMREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBMREF_OK = 0,
    LBMREF_ERR_INVALID_ARG = -1,
    LBMREF_ERR_DOMAIN = -2 /* psi^2 < 0, rho <= 0, b*rho >= 1 or non-finite */
};

typedef struct {
    int32_t nx, ny;       /* periodic lattice, >= 3 each                      */
    double tau;           /* BGK relaxation time, Eq. BGKCO                   */
    double G;             /* pseudopotential sign / scale, Eq. DED            */
    double epsilon;       /* coexistence parameter of Eq. IFT                 */
    double sigma;         /* surface-tension parameter of Eq. IFT             */
    double eos_a, eos_b, eos_c, eos_k, T; /* Carnahan-Starling, Eq. CSEOS     */
    int32_t force_on;     /* 0: F = 0 (plain BGK); 1: the force of Eq. IFT    */
    int32_t m2_trace_alt; /* 0: direct trace of Eq. SOMED; 1: 2 cs^2 (M0-psi) */
    int32_t storage;      /* 0: exact FP64 state; 1, 2: the state is kept as
                             deviations f_i - w_i rho_ref rounded to IEEE
                             binary32 (1) or binary16 (2) after every step and
                             at initialisation (reduced-precision storage);
                             3: per source cell z, the nine post-collision
                             values are kept as binary16 deviations
                             X_i = round16(f*_i - w_i R) from w_i times the
                             cell's own FP32 reference R = sum_i f*_i, with R
                             then corrected by the rounding errors,
                             R <- round32(R + sum_i (f*_i - w_i R - X_i)), so
                             that sum_i (X_i + w_i R) keeps the cell's mass;
                             f*_i becomes X_i + w_i R                           */
    double rho_ref;       /* reference density of the stored deviations       */
    int32_t collision;    /* 0: BGK (Eq. BGKCO) with the Guo factor of
                             Eq. GFSBGK; 1: MRT (Eq. MRTCO) with the Guo
                             factor of Eq. GFSMRT, moment matrix of
                             Eq. MatrixMRT (Appendix A)                        */
    double tau_rho, tau_e, tau_zeta, tau_j, tau_q; /* MRT relaxation times of
                             Eq. RelaxationMatrix; the stress rows relax with
                             tau_nu = tau.  Ignored for BGK.                   */
} lbmref_params;

/* Diagnostic record of the first domain failure (cell = y*nx + x). */
typedef struct {
    int64_t step; /* number of completed steps when the failure was found */
    int64_t cell;
    double rho;
} lbmref_fault;

/* Pointwise building blocks. */
double lbmref_eos_pressure(const lbmref_params *p, double rho);          /* Eq. CSEOS */
int lbmref_psi(const lbmref_params *p, double rho, double *psi);          /* Eq. DED   */
void lbmref_equilibrium(double rho, double ux, double uy, double feq[9]); /* Eq. SEDF  */
void lbmref_guo_source(double tau, double ux, double uy, double Fx, double Fy,
                       double S[9]);                                      /* Eqs. GFS, GFSBGK */
/* The bracket of Eq. GFS without C_ij:
 * s_j = w_j [ c_ja F_a / cs^2 + (c_ja c_jb - cs^2 d_ab) F_a u_b / cs^4 ]. */
void lbmref_guo_term(double ux, double uy, double Fx, double Fy, double s[9]);
/* The moment matrix M of Eq. MatrixMRT, row-major (M[9 k + i] = M_ki). */
void lbmref_mrt_matrix(double M[81]);
/* The MRT collision matrices of the parameters: K = M^-1 Lambda M
 * (Eq. MRTCO) and C = M^-1 (I - Lambda/2) M (Eq. GFSMRT), row-major, with
 * M^-1 from Gauss-Jordan elimination.  Returns LBMREF_ERR_INVALID_ARG for
 * invalid parameters. */
int lbmref_mrt_operators(const lbmref_params *p, double K[81], double C[81]);

/* Field operations over a periodic psi field [ny][nx]. */
void lbmref_psi_moments(int32_t nx, int32_t ny, const double *psi, double *M0,
                        double *M1x, double *M1y, double *M2xx, double *M2xy,
                        double *M2yy);                     /* Eqs. ZOMED, FOMED, SOMED */
void lbmref_force(const lbmref_params *p, const double *psi, double *Fx,
                  double *Fy);                            /* Eq. IFT, moment form      */
void lbmref_force_aij(const lbmref_params *p, const double *psi, double *Fx,
                      double *Fy);                        /* Eq. Ansatz with A_ij      */

/* Lattice operations. */
int lbmref_init(const lbmref_params *p, const double *rho0, const double *ux0,
                const double *uy0, double *f);            /* f(0) = f^eq(rho0, u0)     */
int lbmref_moments(const lbmref_params *p, const double *f, double *rho,
                   double *ux, double *uy, double *Fx, double *Fy, double *psi,
                   lbmref_fault *fault);                  /* Eqs. FD, FMD at time t    */
int lbmref_step(const lbmref_params *p, double *f, int64_t nsteps,
                lbmref_fault *fault);                     /* Eq. TLBE, nsteps times    */
int lbmref_threads(void);                                  /* OpenMP threads it will use */
void lbmref_set_threads(int n);                            /* use n > 0 threads from now on */

/* Round x to the nearest value of the storage format (ties to even):
 * 0 -> x unchanged, 1 -> IEEE binary32, 2 -> IEEE binary16 (with subnormals,
 * overflow to infinity). */
double lbmref_quantize(int32_t storage, double x);

#ifdef __cplusplus
}
#endif

#endif /* LBMREF_H */
