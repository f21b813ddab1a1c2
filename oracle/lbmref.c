/*
 * lbmref.c -- plain FP64 CPU oracle for the D2Q9 force-approach
 * pseudopotential lattice Boltzmann update of arXiv:2003.07968.
 *
 * TEST INFRASTRUCTURE ONLY: see lbmref.h.  Nothing here is tuned.  Every step
 * is a separate full-lattice phase, sums run in the order the equations are
 * written, and c_s^2 stays a symbol (CS2) so each line can be read against
 * the paper.  Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp.
 */
#include "lbmref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* D2Q9 velocity set, Sec. II.A (Eq. VelocitySet). */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* Weights and sound speed, Sec. II.A below Eq. SEDF. */
static const double W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                            1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
#define CS2 (1.0 / 3.0)

static double c_comp(int i, int a) { return a == 0 ? (double)CX[i] : (double)CY[i]; }
static double kdelta(int a, int b) { return a == b ? 1.0 : 0.0; }
static int wrap(int v, int n) { return ((v % n) + n) % n; }

int lbmref_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void lbmref_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Rounding to the storage formats.  binary16 has 11 significant bits, normal
 * numbers from 2^-14 to 65504 and subnormals spaced 2^-24; values from 65520
 * up round to infinity.  The spacing of representable values around |x| is
 * 2^(e - 11) for |x| in [2^(e-1), 2^e), never below 2^-24, so rounding is a
 * scaling by a power of two, an integer round (ties to even) and the scaling
 * back, all exact except the round itself. */
static double round_binary16(double x)
{
    if (!isfinite(x) || x == 0.0) return x;
    double a = fabs(x);
    if (a >= 65520.0) return copysign(INFINITY, x);
    int e;
    frexp(a, &e);
    int ulp_exp = e - 11;
    if (ulp_exp < -24) ulp_exp = -24;
    double r = nearbyint(ldexp(a, -ulp_exp));
    return copysign(ldexp(r, ulp_exp), x);
}

double lbmref_quantize(int32_t storage, double x)
{
    if (storage == 1) return (double)(float)x;
    if (storage == 2) return round_binary16(x);
    return x;
}

/* Storage mode 3: the nine values f[i * n + k] that cell k sends are kept as
 * binary16 deviations from w_i R with R = sum_i f_i, R corrected by the
 * rounding errors and rounded to binary32. */
static void store_round_local(double *f, size_t n)
{
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < n; ++k) {
        double R = 0.0;
        for (int i = 0; i < 9; ++i)
            R += f[(size_t)i * n + k];
        double X[9], err = 0.0;
        for (int i = 0; i < 9; ++i) {
            double dev = f[(size_t)i * n + k] - W[i] * R;
            X[i] = lbmref_quantize(2, dev);
            err += dev - X[i];
        }
        double Rs = lbmref_quantize(1, R + err);
        for (int i = 0; i < 9; ++i)
            f[(size_t)i * n + k] = X[i] + W[i] * Rs;
    }
}

/* Reduced-precision storage: f_i = w_i rho_ref + round(f_i - w_i rho_ref), or
 * the per-cell form of mode 3.  f holds post-collision values indexed by the
 * cell that sends them. */
static void store_round(const lbmref_params *p, double *f, size_t n)
{
    if (!p->storage) return;
    if (p->storage == 3) {
        store_round_local(f, n);
        return;
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < 9; ++i)
        for (size_t k = 0; k < n; ++k) {
            double base = W[i] * p->rho_ref;
            f[(size_t)i * n + k] = base + lbmref_quantize(p->storage, f[(size_t)i * n + k] - base);
        }
}

/* Carnahan-Starling equation of state, Sec. IV.A (Eq. CSEOS):
 * P = k [ c rho T (1 + b rho + (b rho)^2 - (b rho)^3) / (1 - b rho)^3 - a rho^2 ]. */
double lbmref_eos_pressure(const lbmref_params *p, double rho)
{
    double br = p->eos_b * rho;
    double num = 1.0 + br + br * br - br * br * br;
    double den = (1.0 - br) * (1.0 - br) * (1.0 - br);
    return p->eos_k * (p->eos_c * rho * p->T * num / den - p->eos_a * rho * rho);
}

/* Pseudopotential from the EOS, Sec. II.B (Eq. DED): psi = sqrt((P - cs^2 rho)/G).
 * The domain is rho > 0, b rho < 1 and a non-negative, finite radicand; the
 * oracle never clamps. */
int lbmref_psi(const lbmref_params *p, double rho, double *psi)
{
    if (!(rho > 0.0) || !(p->eos_b * rho < 1.0) || !isfinite(rho))
        return LBMREF_ERR_DOMAIN;
    double radicand = (lbmref_eos_pressure(p, rho) - CS2 * rho) / p->G;
    if (!(radicand >= 0.0) || !isfinite(radicand))
        return LBMREF_ERR_DOMAIN;
    *psi = sqrt(radicand);
    return LBMREF_OK;
}

/* Second-order equilibrium, Sec. II.A (Eq. SEDF):
 * f_i^eq = w_i [ rho + c_ia rho u_a / cs^2 + (c_ia c_ib - cs^2 d_ab) rho u_a u_b / (2 cs^4) ]. */
void lbmref_equilibrium(double rho, double ux, double uy, double feq[9])
{
    double u[2] = {ux, uy};
    for (int i = 0; i < 9; ++i) {
        double lin = 0.0, quad = 0.0;
        for (int a = 0; a < 2; ++a)
            lin += c_comp(i, a) * rho * u[a] / CS2;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                quad += (c_comp(i, a) * c_comp(i, b) - CS2 * kdelta(a, b)) * rho * u[a] *
                        u[b] / (2.0 * CS2 * CS2);
        feq[i] = W[i] * (rho + lin + quad);
    }
}

/* Guo source with the BGK factor, Sec. II.A (Eqs. GFS, GFSBGK):
 * S_i = (1 - 1/(2 tau)) w_i [ c_ia F_a / cs^2 + (c_ia c_ib - cs^2 d_ab) F_a u_b / cs^4 ]. */
void lbmref_guo_source(double tau, double ux, double uy, double Fx, double Fy, double S[9])
{
    double u[2] = {ux, uy};
    double F[2] = {Fx, Fy};
    for (int i = 0; i < 9; ++i) {
        double lin = 0.0, quad = 0.0;
        for (int a = 0; a < 2; ++a)
            lin += c_comp(i, a) * F[a] / CS2;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                quad += (c_comp(i, a) * c_comp(i, b) - CS2 * kdelta(a, b)) * F[a] * u[b] /
                        (CS2 * CS2);
        S[i] = (1.0 - 1.0 / (2.0 * tau)) * W[i] * (lin + quad);
    }
}

void lbmref_guo_term(double ux, double uy, double Fx, double Fy, double s[9])
{
    double u[2] = {ux, uy};
    double F[2] = {Fx, Fy};
    for (int i = 0; i < 9; ++i) {
        double lin = 0.0, quad = 0.0;
        for (int a = 0; a < 2; ++a)
            lin += c_comp(i, a) * F[a] / CS2;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                quad += (c_comp(i, a) * c_comp(i, b) - CS2 * kdelta(a, b)) * F[a] * u[b] /
                        (CS2 * CS2);
        s[i] = W[i] * (lin + quad);
    }
}

/* Gram-Schmidt moment matrix of Appendix A (Eq. MatrixMRT); rows are the
 * moments rho, e, zeta, j_x, q_x, j_y, q_y, p_xx, p_xy. */
static const double MRT_M[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
};

void lbmref_mrt_matrix(double M[81])
{
    for (int k = 0; k < 9; ++k)
        for (int i = 0; i < 9; ++i)
            M[9 * k + i] = MRT_M[k][i];
}

/* Inverse of a 9 x 9 matrix by Gauss-Jordan elimination with partial
 * pivoting; returns -1 if it is singular. */
static int invert9(const double A[81], double Ainv[81])
{
    double a[9][18];
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 18; ++c)
            a[r][c] = c < 9 ? A[9 * r + c] : (c - 9 == r ? 1.0 : 0.0);
    for (int col = 0; col < 9; ++col) {
        int piv = col;
        for (int r = col + 1; r < 9; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (a[piv][col] == 0.0) return -1;
        if (piv != col)
            for (int c = 0; c < 18; ++c) {
                double t = a[col][c];
                a[col][c] = a[piv][c];
                a[piv][c] = t;
            }
        double d = a[col][col];
        for (int c = 0; c < 18; ++c)
            a[col][c] /= d;
        for (int r = 0; r < 9; ++r)
            if (r != col) {
                double m = a[r][col];
                for (int c = 0; c < 18; ++c)
                    a[r][c] -= m * a[col][c];
            }
    }
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c)
            Ainv[9 * r + c] = a[r][9 + c];
    return 0;
}

static int check_params(const lbmref_params *p);

/* Relaxation matrix of Eq. RelaxationMatrix:
 * Lambda = diag(1/tau_rho, 1/tau_e, 1/tau_zeta, 1/tau_j, 1/tau_q, 1/tau_j,
 *               1/tau_q, 1/tau_nu, 1/tau_nu), tau_nu = tau. */
int lbmref_mrt_operators(const lbmref_params *p, double K[81], double C[81])
{
    int st = check_params(p);
    if (st) return st;
    double M[81], Minv[81];
    lbmref_mrt_matrix(M);
    if (invert9(M, Minv)) return LBMREF_ERR_INVALID_ARG;
    double lam[9] = {1.0 / p->tau_rho, 1.0 / p->tau_e, 1.0 / p->tau_zeta,
                     1.0 / p->tau_j,   1.0 / p->tau_q, 1.0 / p->tau_j,
                     1.0 / p->tau_q,   1.0 / p->tau,   1.0 / p->tau};
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j) {
            double k = 0.0, c = 0.0;
            for (int m = 0; m < 9; ++m) {
                k += Minv[9 * i + m] * lam[m] * M[9 * m + j];
                c += Minv[9 * i + m] * (1.0 - lam[m] / 2.0) * M[9 * m + j];
            }
            K[9 * i + j] = k;
            C[9 * i + j] = c;
        }
    return LBMREF_OK;
}

/* Moments of w_i psi(x + c_i), Sec. III.B (Eqs. ZOMED, FOMED, SOMED). */
static void moments_at(int32_t nx, int32_t ny, const double *psi, int x, int y, double *M0,
                       double M1[2], double M2[2][2])
{
    *M0 = 0.0;
    M1[0] = M1[1] = 0.0;
    M2[0][0] = M2[0][1] = M2[1][0] = M2[1][1] = 0.0;
    for (int i = 0; i < 9; ++i) {
        double v = psi[(size_t)wrap(y + CY[i], ny) * nx + wrap(x + CX[i], nx)];
        *M0 += W[i] * v;
        for (int a = 0; a < 2; ++a)
            M1[a] += W[i] * c_comp(i, a) * v;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                M2[a][b] += W[i] * (c_comp(i, a) * c_comp(i, b) - CS2 * kdelta(a, b)) * v;
    }
}

void lbmref_psi_moments(int32_t nx, int32_t ny, const double *psi, double *M0, double *M1x,
                        double *M1y, double *M2xx, double *M2xy, double *M2yy)
{
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double m0, m1[2], m2[2][2];
            moments_at(nx, ny, psi, x, y, &m0, m1, m2);
            size_t k = (size_t)y * nx + x;
            if (M0) M0[k] = m0;
            if (M1x) M1x[k] = m1[0];
            if (M1y) M1y[k] = m1[1];
            if (M2xx) M2xx[k] = m2[0][0];
            if (M2xy) M2xy[k] = m2[0][1];
            if (M2yy) M2yy[k] = m2[1][1];
        }
}

/* The proposed force, Sec. III.C (Eq. IFT), built from
 *   F^SC_a  = -psi(x) (2G/cs^2) sum_i w_i psi(x+c_i) c_ia        (Eq. SCF)
 *   F^(1)_a = -2 (M1_b/cs^2)(M2_ab/cs^4)                          (Eq. DFTCCC)
 *   F^(2)_a = (M1_a/cs^2)(M2_bb/cs^4) - (M1_b/cs^2)(M2_ab/cs^4)   (Eq. DFTCST)
 *   F_a     = F^SC_a - (3/4) eps cs^2 G F^(1)_a + (sigma - 1) cs^2 G F^(2)_a.
 * M2_bb is the direct trace of Eq. SOMED, or 2 cs^2 (M0 - psi) when
 * m2_trace_alt is set (the alternative stencil stated after Eq. DFTCST). */
static void force_at(const lbmref_params *p, const double *psi, int x, int y, double F[2])
{
    double M0, M1[2], M2[2][2];
    moments_at(p->nx, p->ny, psi, x, y, &M0, M1, M2);
    double psi0 = psi[(size_t)y * p->nx + x];
    double trace = p->m2_trace_alt ? 2.0 * CS2 * (M0 - psi0) : M2[0][0] + M2[1][1];
    for (int a = 0; a < 2; ++a) {
        double fsc = -psi0 * (2.0 * p->G / CS2) * M1[a];
        double f1 = 0.0;
        for (int b = 0; b < 2; ++b)
            f1 += -2.0 * (M1[b] / CS2) * (M2[a][b] / (CS2 * CS2));
        double f2 = (M1[a] / CS2) * (trace / (CS2 * CS2));
        for (int b = 0; b < 2; ++b)
            f2 -= (M1[b] / CS2) * (M2[a][b] / (CS2 * CS2));
        F[a] = fsc - 0.75 * p->epsilon * CS2 * p->G * f1 + (p->sigma - 1.0) * CS2 * p->G * f2;
    }
}

void lbmref_force(const lbmref_params *p, const double *psi, double *Fx, double *Fy)
{
#pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            double F[2];
            force_at(p, psi, x, y, F);
            Fx[(size_t)y * p->nx + x] = F[0];
            Fy[(size_t)y * p->nx + x] = F[1];
        }
}

/* The same force as the double sum of Eq. Ansatz, F_a = sum_ij A_ij psi_i psi_j,
 * with the A_ij tensor given at the end of Sec. III.C.  The Shan-Chen block of
 * that tensor is used with its velocity component c_ia, which the printed
 * expression drops: without it the block is not a vector and does not
 * reproduce Eq. SCF.  The trace term uses d_bb = 2 (two dimensions), so this
 * form corresponds to the direct trace. */
void lbmref_force_aij(const lbmref_params *p, const double *psi, double *Fx, double *Fy)
{
    double k1 = (1.5 * p->epsilon - (p->sigma - 1.0)) * CS2 * p->G;
    double k2 = (p->sigma - 1.0) * CS2 * p->G;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            double F[2] = {0.0, 0.0};
            for (int a = 0; a < 2; ++a)
                for (int i = 0; i < 9; ++i)
                    for (int j = 0; j < 9; ++j) {
                        double wij = W[i] * W[j] / (CS2 * CS2 * CS2);
                        double t1 = 0.0;
                        for (int b = 0; b < 2; ++b)
                            t1 += c_comp(i, b) *
                                  (c_comp(j, a) * c_comp(j, b) - CS2 * kdelta(a, b));
                        double cjcj = c_comp(j, 0) * c_comp(j, 0) + c_comp(j, 1) * c_comp(j, 1);
                        double t2 = c_comp(i, a) * (cjcj - CS2 * 2.0);
                        double A = -(2.0 * p->G / CS2) * W[i] * c_comp(i, a) * (j == 0 ? 1.0 : 0.0) +
                                   k1 * wij * t1 + k2 * wij * t2;
                        double pi = psi[(size_t)wrap(y + CY[i], p->ny) * p->nx +
                                        wrap(x + CX[i], p->nx)];
                        double pj = psi[(size_t)wrap(y + CY[j], p->ny) * p->nx +
                                        wrap(x + CX[j], p->nx)];
                        F[a] += A * pi * pj;
                    }
            Fx[(size_t)y * p->nx + x] = F[0];
            Fy[(size_t)y * p->nx + x] = F[1];
        }
}

static int check_params(const lbmref_params *p)
{
    if (!p || p->nx < 3 || p->ny < 3) return LBMREF_ERR_INVALID_ARG;
    if (!(p->tau > 0.5) || !isfinite(p->tau)) return LBMREF_ERR_INVALID_ARG;
    if (!(p->G != 0.0) || !isfinite(p->G)) return LBMREF_ERR_INVALID_ARG;
    if (p->storage < 0 || p->storage > 3 || !isfinite(p->rho_ref)) return LBMREF_ERR_INVALID_ARG;
    if (p->collision != 0 && p->collision != 1) return LBMREF_ERR_INVALID_ARG;
    if (p->collision == 1) {
        const double taus[5] = {p->tau_rho, p->tau_e, p->tau_zeta, p->tau_j, p->tau_q};
        for (int k = 0; k < 5; ++k)
            if (!(taus[k] > 0.5) || !isfinite(taus[k])) return LBMREF_ERR_INVALID_ARG;
    }
    return LBMREF_OK;
}

/* Initial state, Sec. IV.A below Eq. ISD: f_i(t=0) = f_i^eq(rho0, u0). */
int lbmref_init(const lbmref_params *p, const double *rho0, const double *ux0,
                const double *uy0, double *f)
{
    int st = check_params(p);
    if (st) return st;
    size_t n = (size_t)p->nx * p->ny;
    for (size_t k = 0; k < n; ++k) {
        double feq[9];
        lbmref_equilibrium(rho0[k], ux0 ? ux0[k] : 0.0, uy0 ? uy0[k] : 0.0, feq);
        for (int i = 0; i < 9; ++i)
            f[(size_t)i * n + k] = feq[i];
    }
    if (p->storage == 3) {
        /* group the values by the cell z = x - c_i that streams them to x */
        double *g = malloc(9 * n * sizeof(double));
        if (!g) return LBMREF_ERR_INVALID_ARG;
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x)
                for (int i = 0; i < 9; ++i)
                    g[(size_t)i * n + (size_t)y * p->nx + x] =
                        f[(size_t)i * n + (size_t)wrap(y + CY[i], p->ny) * p->nx +
                          wrap(x + CX[i], p->nx)];
        store_round(p, g, n);
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x)
                for (int i = 0; i < 9; ++i)
                    f[(size_t)i * n + (size_t)wrap(y + CY[i], p->ny) * p->nx +
                      wrap(x + CX[i], p->nx)] = g[(size_t)i * n + (size_t)y * p->nx + x];
        free(g);
        return LBMREF_OK;
    }
    store_round(p, f, n);
    return LBMREF_OK;
}

/* Density (Eq. FD), pseudopotential (Eq. DED), force (Eq. IFT or zero) and
 * velocity (Eq. FMD: rho u = sum_i f_i c_i + F/2) of the state f, as separate
 * full-lattice phases.  Returns LBMREF_ERR_DOMAIN at the first cell (in index
 * order) whose density leaves the EOS domain. */
static int macroscopic(const lbmref_params *p, const double *f, double *rho, double *psi,
                       double *Fx, double *Fy, double *ux, double *uy, int64_t *bad_cell)
{
    size_t n = (size_t)p->nx * p->ny;
    int nx = p->nx, ny = p->ny;
    int *row_bad = malloc((size_t)ny * sizeof(int));
    if (!row_bad) return LBMREF_ERR_INVALID_ARG;
    /* phase: density */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t k = (size_t)y * nx + x;
            double s = 0.0;
            for (int i = 0; i < 9; ++i)
                s += f[(size_t)i * n + k];
            rho[k] = s;
        }
    /* phase: pseudopotential (or, with the force off, only the density check) */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        row_bad[y] = -1;
        for (int x = 0; x < nx; ++x) {
            size_t k = (size_t)y * nx + x;
            int ok;
            if (p->force_on) {
                ok = lbmref_psi(p, rho[k], &psi[k]) == LBMREF_OK;
            } else {
                ok = rho[k] > 0.0 && isfinite(rho[k]);
                psi[k] = 0.0;
            }
            if (!ok && row_bad[y] < 0) row_bad[y] = x;
        }
    }
    for (int y = 0; y < ny; ++y)
        if (row_bad[y] >= 0) {
            *bad_cell = (int64_t)y * nx + row_bad[y];
            free(row_bad);
            return LBMREF_ERR_DOMAIN;
        }
    free(row_bad);
    /* phase: force */
    if (p->force_on) {
        lbmref_force(p, psi, Fx, Fy);
    } else {
        for (size_t k = 0; k < n; ++k) {
            Fx[k] = 0.0;
            Fy[k] = 0.0;
        }
    }
    /* phase: velocity */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t k = (size_t)y * nx + x;
            double m[2] = {0.0, 0.0};
            for (int i = 0; i < 9; ++i)
                for (int a = 0; a < 2; ++a)
                    m[a] += f[(size_t)i * n + k] * c_comp(i, a);
            ux[k] = (m[0] + Fx[k] / 2.0) / rho[k];
            uy[k] = (m[1] + Fy[k] / 2.0) / rho[k];
        }
    return LBMREF_OK;
}

int lbmref_moments(const lbmref_params *p, const double *f, double *rho, double *ux,
                   double *uy, double *Fx, double *Fy, double *psi, lbmref_fault *fault)
{
    int st = check_params(p);
    if (st) return st;
    int64_t bad = -1;
    st = macroscopic(p, f, rho, psi, Fx, Fy, ux, uy, &bad);
    if (st && fault) {
        fault->step = 0;
        fault->cell = bad;
        fault->rho = rho[bad];
    }
    return st;
}

/* One lattice Boltzmann step per Eq. TLBE with the BGK operator (Eq. BGKCO)
 * and the Guo source (Eqs. GFS, GFSBGK):
 *   f*_i(x) = f_i(x) - (f_i(x) - f_i^eq(x))/tau + S_i(x)     (collision)
 *   f_i(x + c_i, t + 1) = f*_i(x)                          (streaming)
 * or, with collision = 1, the MRT operator (Eq. MRTCO) and the MRT Guo
 * factor (Eq. GFSMRT):
 *   f*_i(x) = f_i - sum_j K_ij (f_j - f_j^eq) + sum_j C_ij s_j
 * with K = M^-1 Lambda M, C = M^-1 (I - Lambda/2) M and s the bracket of
 * Eq. GFS; f^eq and s evaluated at the velocity of Eq. FMD. */
int lbmref_step(const lbmref_params *p, double *f, int64_t nsteps, lbmref_fault *fault)
{
    int st = check_params(p);
    if (st) return st;
    if (nsteps < 0) return LBMREF_ERR_INVALID_ARG;
    size_t n = (size_t)p->nx * p->ny;
    double *rho = malloc(n * sizeof(double));
    double *psi = malloc(n * sizeof(double));
    double *Fx = malloc(n * sizeof(double));
    double *Fy = malloc(n * sizeof(double));
    double *ux = malloc(n * sizeof(double));
    double *uy = malloc(n * sizeof(double));
    double *fpost = malloc(9 * n * sizeof(double));
    if (!rho || !psi || !Fx || !Fy || !ux || !uy || !fpost) {
        st = LBMREF_ERR_INVALID_ARG;
        goto done;
    }
    double K[81], C[81];
    if (p->collision == 1) {
        st = lbmref_mrt_operators(p, K, C);
        if (st) goto done;
    }
    for (int64_t t = 0; t < nsteps; ++t) {
        int64_t bad = -1;
        st = macroscopic(p, f, rho, psi, Fx, Fy, ux, uy, &bad);
        if (st) {
            if (fault) {
                fault->step = t;
                fault->cell = bad;
                fault->rho = rho[bad];
            }
            goto done;
        }
        /* phase: collision */
#pragma omp parallel for schedule(static)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                size_t k = (size_t)y * p->nx + x;
                double feq[9], S[9];
                lbmref_equilibrium(rho[k], ux[k], uy[k], feq);
                if (p->collision == 1) {
                    double s[9], neq[9];
                    lbmref_guo_term(ux[k], uy[k], Fx[k], Fy[k], s);
                    for (int j = 0; j < 9; ++j)
                        neq[j] = f[(size_t)j * n + k] - feq[j];
                    for (int i = 0; i < 9; ++i) {
                        double relax = 0.0, src = 0.0;
                        for (int j = 0; j < 9; ++j) {
                            relax += K[9 * i + j] * neq[j];
                            src += C[9 * i + j] * s[j];
                        }
                        fpost[(size_t)i * n + k] = f[(size_t)i * n + k] - relax + src;
                    }
                    continue;
                }
                lbmref_guo_source(p->tau, ux[k], uy[k], Fx[k], Fy[k], S);
                for (int i = 0; i < 9; ++i) {
                    double fi = f[(size_t)i * n + k];
                    fpost[(size_t)i * n + k] = fi - (fi - feq[i]) / p->tau + S[i];
                }
            }
        /* phase: storage rounding (reduced-precision storage only) */
        store_round(p, fpost, n);
        /* phase: streaming, periodic */
#pragma omp parallel for schedule(static)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x)
                for (int i = 0; i < 9; ++i) {
                    size_t dst = (size_t)wrap(y + CY[i], p->ny) * p->nx + wrap(x + CX[i], p->nx);
                    f[(size_t)i * n + dst] = fpost[(size_t)i * n + (size_t)y * p->nx + x];
                }
    }
done:
    free(rho);
    free(psi);
    free(Fx);
    free(Fy);
    free(ux);
    free(uy);
    free(fpost);
    return st;
}
