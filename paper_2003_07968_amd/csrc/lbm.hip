// lbm.hip -- D2Q9 force-approach pseudopotential lattice Boltzmann update for
// AMD CDNA4 (gfx950), behind the C ABI of include/lbm.h.
//
// Method: Czelusniak et al., arXiv:2003.07968.  Per cell and step: pull
// streaming (Eq. TLBE), density (Eq. FD), Carnahan-Starling pressure
// (Eq. CSEOS), pseudopotential (Eq. DED), psi moments (Eqs. FOMED, SOMED), the
// proposed force (Eq. IFT), velocity (Eq. FMD) and the Guo-forced BGK
// collision (Eqs. BGKCO, SEDF, GFS, GFSBGK), or the multiple-relaxation-time
// collision with the Guo source in moment space (Eqs. MRTCO, GFSMRT, the
// Gram-Schmidt moment matrix of Eq. MatrixMRT).
//
// Storage modes: FP64 populations with FP64 arithmetic, or populations kept
// as deviations d_i = f_i - w_i rho_ref in FP32 or FP16 with FP32 arithmetic
// (rho_ref is a reference density, normally the mean), or as FP16 deviations
// from w_i R(z) with a per-cell FP32 reference R (the nine values a cell sends
// share its R).  The diagnostics reductions are FP64 in every mode.
//
// Kernel design (one fused pass per step, or per two steps):
//   * populations are arrays X_i[y][x] holding the post-collision values of
//     the previous step; the pulled value is f_i(x) = X_i(x - c_i), so every
//     row is read with unit stride (shifted by at most one element) and
//     written with unit stride.  The nine rows X_0[y] .. X_8[y] of one y are
//     stored one after another (row-interleaved), so that a row step reads
//     and writes three neighbouring blocks of memory instead of nine regions
//     a whole plane apart;
//   * single step: a workgroup of BX threads owns a strip of interior columns
//     (BX - 2, rounded down to a multiple of 128 bytes) plus one halo column
//     on each side, and walks a segment of rows.  At each row it loads the
//     pulled populations of the row ahead, turns them into rho and psi,
//     exchanges psi with its x-neighbours through one double-buffered LDS
//     row, and keeps the 3x3 psi window of its own column in registers;
//     populations are prefetched one further row ahead.  Each population is
//     read from HBM once per step, apart from the halo columns and rows,
//     which are re-read through L2; neighbouring segments walk in opposite
//     directions, so both workgroups of a segment boundary touch its rows at
//     about the same time;
//   * two steps per pass (the default): the first step is computed on a tile
//     widened by three columns and rows on each side and handed to the
//     second through LDS, so the populations are read and written once per
//     two updates (walk2 below);
//   * workgroups take their tiles in an XCD-aware order (xcd_tile).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "lbm.h"

namespace {

constexpr int kQ = 9;
constexpr int kMaxTiles = 1 << 15; // bound on workgroups per sweep (sizes the scratch)
constexpr int kDiag = 6;          // diagnostics values per workgroup
#ifndef LBM_PREFETCH
#define LBM_PREFETCH 1
#endif
constexpr int kPrefetch = LBM_PREFETCH; // rows in flight beyond the leading row (step sweep)
constexpr size_t kAlign = 256;

// Storage formats of the populations and the arithmetic type used with them.
template <int ST> struct Store;
template <> struct Store<LBM_STORE_F64> {
    using E = double;  // stored element
    using R = double;  // arithmetic
    static constexpr bool local = false;  // per-cell reference density
};
template <> struct Store<LBM_STORE_F32_SHIFTED> {
    using E = float;
    using R = float;
    static constexpr bool local = false;
};
template <> struct Store<LBM_STORE_F16_SHIFTED> {
    using E = _Float16;
    using R = float;
    static constexpr bool local = false;
};
template <> struct Store<LBM_STORE_F16_LOCAL> {
    using E = _Float16;
    using R = float;
    static constexpr bool local = true;
};

size_t elem_size(int storage)
{
    return storage == LBM_STORE_F64 ? 8 : (storage == LBM_STORE_F32_SHIFTED ? 4 : 2);
}

bool is_f16(int storage)
{
    return storage == LBM_STORE_F16_SHIFTED || storage == LBM_STORE_F16_LOCAL;
}

// Coefficients of one lattice, precomputed on the host.
struct Coeffs {
    int nx, ny;
    int pitch;      // stride between rows y and y + 1 of one population, in elements
    size_t plane;   // stride between populations i and i + 1 of one row, in elements
    double omega;   // 1/tau
    double guo;     // 1 - 1/(2 tau), Eq. GFSBGK
    double eos_b;   // b of Eq. CSEOS
    double kcT;     // k c T
    double ka;      // k a
    double invG;    // 1/G
    // Eq. IFT with cs^2 = 1/3 substituted:
    //   F_a = cSC psi0 M1_a + cA (M1_b M2_ab) + cB M1_a M2_bb
    // cSC = -2G/cs^2 = -6G; cA = (3/2 eps - (sigma - 1)) cs^2 G / cs^6
    // = 9G (1.5 eps - sigma + 1); cB = (sigma - 1) cs^2 G / cs^6 = 9G (sigma - 1).
    double cSC, cA, cB;
    double rho_ref; // populations are stored as f_i - w_i rho_ref (0 for FP64 and the
                    // per-cell mode)
    size_t r_off;   // per-cell mode: byte offset of the FP32 reference block in a buffer
    int r_pitch;    // per-cell mode: row pitch of that block, in floats
    double s_e, s_z, s_q; // MRT rates 1/tau_e, 1/tau_zeta, 1/tau_q (the stress rows use omega)
    int coll;       // lbm_collision
    int force_on;
    int trace_alt;
    int storage;
};

// The coefficients in the arithmetic type of a storage mode.
template <class R>
struct Phys {
    R omega, guo, eos_b, kcT, ka, invG, cSC, cA, cB, rho_ref, s_e, s_z, s_q;
    int trace_alt;
    __device__ explicit Phys(const Coeffs &c)
        : omega((R)c.omega), guo((R)c.guo), eos_b((R)c.eos_b), kcT((R)c.kcT), ka((R)c.ka),
          invG((R)c.invG), cSC((R)c.cSC), cA((R)c.cA), cB((R)c.cB), rho_ref((R)c.rho_ref),
          s_e((R)c.s_e), s_z((R)c.s_z), s_q((R)c.s_q), trace_alt(c.trace_alt)
    {
    }
};

// Tile decomposition of one sweep.  Strip s covers interior columns
// [s * width, min(nx, (s + 1) * width)); width is a multiple of the storage's
// store alignment (64-128 bytes) whenever the lattice needs more than one
// strip, so the stores of neighbouring workgroups never share a cache line.
struct Tiles {
    int nstrips, nseg, ntiles, width;
};

// Optional outputs of the moments sweep.
struct Fields {
    double *rho, *ux, *uy, *Fx, *Fy, *psi;
};

enum Mode { kStep = 0, kMoments = 1, kDiagnostics = 2 };

__device__ __forceinline__ int wrap_lo(int v, int n) { return v < 0 ? v + n : v; }
__device__ __forceinline__ int wrap_hi(int v, int n) { return v >= n ? v - n : v; }

// Pulled populations of row r at column x: f_i(x, r) = X_i(x - c_ix, r - c_iy).
// Row bases are uniform across the workgroup (scalar registers) and the
// column enters as a 32-bit byte offset, so each load is a single
// scalar-base + vector-offset global load.
struct Cols {
    uint32_t o, m, p;  // byte offsets of columns x, x - 1 (wrapped), x + 1 (wrapped)
};

template <class E, class R>
__device__ __forceinline__ R ld(const E *__restrict__ row, uint32_t byte_off)
{
    return (R) * (const E *)((const char *)row + byte_off);
}

// The stored values X_i of the pulled populations, as R.  For the shifted
// modes they are the deviations d_i = f_i - w_i rho_ref (rho_ref = 0 for
// FP64); the per-cell mode turns them into deviations with reconstruct().
template <int ST, class E = typename Store<ST>::E, class R = typename Store<ST>::R>
__device__ __forceinline__ void load_pulled(const E *__restrict__ src, const Coeffs &c, int r,
                                            const Cols &x, R d[kQ])
{
    const int rm = wrap_lo(r - 1, c.ny), rp = wrap_hi(r + 1, c.ny);
    const size_t P = c.plane;
    const E *row_r = src + (size_t)r * c.pitch;
    const E *row_m = src + (size_t)rm * c.pitch;
    const E *row_p = src + (size_t)rp * c.pitch;
    d[0] = ld<E, R>(row_r, x.o);
    d[1] = ld<E, R>(row_r + 1 * P, x.m);
    d[2] = ld<E, R>(row_m + 2 * P, x.o);
    d[3] = ld<E, R>(row_r + 3 * P, x.p);
    d[4] = ld<E, R>(row_p + 4 * P, x.o);
    d[5] = ld<E, R>(row_m + 5 * P, x.m);
    d[6] = ld<E, R>(row_m + 6 * P, x.p);
    d[7] = ld<E, R>(row_p + 7 * P, x.p);
    d[8] = ld<E, R>(row_p + 8 * P, x.m);
}

// R at columns x - 1, x, x + 1 of one lattice row.
template <class R>
struct Tri {
    R l, o, r;
};

// Per-cell mode: the FP32 reference R of lattice row r at column x, and at
// x - 1 for the first lane of the workgroup (its left neighbour is in no lane)
// or x + 1 for every other lane (columns of R are twice as wide as those of
// the binary16 populations).
template <class R>
struct RefPair {
    R own, side;
};

template <class R>
__device__ __forceinline__ RefPair<R> load_ref(const void *__restrict__ src, const Coeffs &c,
                                               int r, const Cols &x, bool first)
{
    const float *row = (const float *)((const char *)src + c.r_off) + (size_t)r * c.r_pitch;
    return RefPair<R>{ld<float, R>(row, 2 * x.o), ld<float, R>(row, 2 * (first ? x.m : x.p))};
}

// Per-cell mode: f_i = X_i + w_i R at the sending cell x - c_i, turned into
// deviations from the cell's own reference, d_i = X_i + w_i (R(x - c_i) - R(x)),
// so that every FP32 operation works on small numbers.  D, C, U hold R of the
// lattice rows r - 1, r, r + 1.
template <class R>
__device__ __forceinline__ void reconstruct(R d[kQ], const Tri<R> &D, const Tri<R> &C,
                                            const Tri<R> &U)
{
    const R w1 = R(1.0 / 9.0), w2 = R(1.0 / 36.0), ref = C.o;
    d[1] = fma(w1, C.l - ref, d[1]);
    d[2] = fma(w1, D.o - ref, d[2]);
    d[3] = fma(w1, C.r - ref, d[3]);
    d[4] = fma(w1, U.o - ref, d[4]);
    d[5] = fma(w2, D.l - ref, d[5]);
    d[6] = fma(w2, D.r - ref, d[6]);
    d[7] = fma(w2, U.r - ref, d[7]);
    d[8] = fma(w2, U.l - ref, d[8]);
}

// Reciprocal and square root in the arithmetic type: IEEE-rounded in FP64 (the
// reference path); the hardware's single-instruction forms in FP32, whose
// error of about one ulp is far below the storage rounding of the
// reduced-precision modes.
__device__ __forceinline__ double recip(double v) { return 1.0 / v; }
__device__ __forceinline__ float recip(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double quot(double a, double b) { return a / b; }
__device__ __forceinline__ float quot(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double root(double v) { return sqrt(v); }
__device__ __forceinline__ float root(float v) { return __builtin_amdgcn_sqrtf(v); }

// Density (Eq. FD) and pseudopotential (Eqs. CSEOS, DED) from the stored
// deviations d_i = f_i - w_i rho_ref: rho = rho_ref + sum_i d_i.  Returns
// false when the density is outside the EOS domain (with FORCE = 0, when it
// is not positive and finite).
template <int FORCE, class R>
__device__ __forceinline__ bool rho_psi(const R d[kQ], R ref, const Phys<R> &P, R &rho, R &psi)
{
    rho = ((((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7]))) + d[8]) + ref;
    if (!FORCE) {
        psi = R(0);
        return rho > R(0) && rho < R(INFINITY);
    }
    const R br = P.eos_b * rho;
    const R num = fma(br, fma(br, R(1) - br, R(1)), R(1));  // 1 + br + br^2 - br^3
    const R om = R(1) - br;
    const R pr = fma(P.kcT * rho, quot(num, om * om * om), -P.ka * rho * rho);
    const R rad = fma(rho, R(-1.0 / 3.0), pr) * P.invG;
    psi = root(rad);
    return rho > R(0) && br < R(1) && rad >= R(0) && rad < R(INFINITY);
}

// Error key of a cell: steps first, then the cell index, so that the
// smallest key is the first failure in the order the oracle reports it.
__device__ __forceinline__ unsigned long long domain_key(long long t, int r, int x, int nx)
{
    return ((unsigned long long)t << 32) | (unsigned long long)((size_t)r * nx + x);
}

// Force of Eq. IFT from s_i = psi(x + c_i) (Eqs. FOMED, SOMED, SCF,
// DFTCCC, DFTCST).
template <class R>
__device__ __forceinline__ void force(const R s[kQ], const Phys<R> &P, R &Fx, R &Fy)
{
    const R d13 = s[1] - s[3], d24 = s[2] - s[4];
    const R s13 = s[1] + s[3], s24 = s[2] + s[4];
    const R a58 = s[5] - s[7], b68 = s[6] - s[8];
    const R s58 = (s[5] + s[6]) + (s[7] + s[8]);
    const R M1x = d13 * R(1.0 / 9.0) + (a58 - b68) * R(1.0 / 36.0);
    const R M1y = d24 * R(1.0 / 9.0) + (a58 + b68) * R(1.0 / 36.0);
    const R M2xx = s[0] * R(-4.0 / 27.0) + s13 * R(2.0 / 27.0) - s24 * R(1.0 / 27.0) +
                   s58 * R(1.0 / 54.0);
    const R M2yy = s[0] * R(-4.0 / 27.0) - s13 * R(1.0 / 27.0) + s24 * R(2.0 / 27.0) +
                   s58 * R(1.0 / 54.0);
    const R M2xy = ((s[5] + s[7]) - (s[6] + s[8])) * R(1.0 / 36.0);
    const R M0 = s[0] * R(4.0 / 9.0) + (s13 + s24) * R(1.0 / 9.0) + s58 * R(1.0 / 36.0);
    const R tr = P.trace_alt ? R(2.0 / 3.0) * (M0 - s[0]) : M2xx + M2yy;
    const R ax = fma(M1x, M2xx, M1y * M2xy);  // (M1 . M2)_x
    const R ay = fma(M1x, M2xy, M1y * M2yy);  // (M1 . M2)_y
    const R sc = P.cSC * s[0], tb = P.cB * tr;
    Fx = fma(sc, M1x, fma(P.cA, ax, tb * M1x));
    Fy = fma(sc, M1y, fma(P.cA, ay, tb * M1y));
}

// Velocity (Eq. FMD).  The w_i rho_ref parts of the populations carry no
// momentum, so the deviations give sum_i f_i c_i directly.
template <class R>
__device__ __forceinline__ void velocity(const R d[kQ], R rho, R Fx, R Fy, R &ux, R &uy)
{
    const R jx = ((d[1] - d[3]) + (d[5] - d[6])) + (d[8] - d[7]);
    const R jy = ((d[2] - d[4]) + (d[5] + d[6])) - (d[7] + d[8]);
    const R inv = recip(rho);
    ux = (jx + R(0.5) * Fx) * inv;
    uy = (jy + R(0.5) * Fy) * inv;
}

// BGK collision with the Guo source (Eqs. BGKCO, SEDF, GFS, GFSBGK), on the
// deviations d_i = f_i - w_i rho_ref, in place:
//   f^eq_i - w_i rho_ref = w_i ((rho - rho_ref) + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u))
//   S_i                  = (1 - 1/(2 tau)) w_i (3 c.F + 9 (c.F)(c.u) - 3 u.F)
//   d_i                 <- d_i + (f^eq_i - w_i rho_ref - d_i)/tau + S_i
// evaluated with the terms of f^eq and S gathered by powers of c_i (below),
// about eight operations per direction.  Multiply-adds are written as
// explicit fma(); the file is compiled without implicit contraction, so every
// inlined copy rounds the same way.
template <class R>
__device__ __forceinline__ void collide(R d[kQ], R ref, R rho, R ux, R uy, R Fx, R Fy,
                                        const Phys<R> &P)
{
    // omega (f^eq_i - w_i rho_ref) + S_i = w_i [A + c_i.B + (c_i.u)(h c_i.u + m c_i.F)]
    // with A = omega (rho (1 - 3/2 u.u) - rho_ref) - 3 g u.F, B = 3 (omega rho u + g F),
    // h = 9/2 omega rho, m = 9 g (g = 1 - 1/(2 tau)); then d_i <- (1 - omega) d_i + w_i [..].
    const R om = P.omega, g = P.guo;
    const R orho = om * rho;
    const R usq = fma(ux, ux, uy * uy);
    const R uF = fma(ux, Fx, uy * Fy);
    const R A = fma(om, fma(rho, R(-1.5) * usq, rho - ref), R(-3) * g * uF);
    const R Bx = R(3) * fma(orho, ux, g * Fx), By = R(3) * fma(orho, uy, g * Fy);
    const R h = R(4.5) * orho;
    const R mx = R(9) * g * Fx, my = R(9) * g * Fy;
    const R keep = R(1) - om;
    const R w0 = R(4.0 / 9.0), w1 = R(1.0 / 9.0), w2 = R(1.0 / 36.0);
    d[0] = fma(keep, d[0], w0 * A);
    const R cu[8] = {ux, uy, -ux, -uy, ux + uy, uy - ux, -ux - uy, ux - uy};
    const R cm[8] = {mx, my, -mx, -my, mx + my, my - mx, -mx - my, mx - my};
    const R cB[8] = {Bx, By, -Bx, -By, Bx + By, By - Bx, -Bx - By, Bx - By};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const R w = k < 4 ? w1 : w2;
        const R q = fma(cu[k], fma(h, cu[k], cm[k]), A + cB[k]);
        d[k + 1] = fma(keep, d[k + 1], w * q);
    }
}

// Multiple-relaxation-time collision with the Guo source (Eqs. MRTCO, GFSMRT)
// on the deviations d_i = f_i - w_i rho_ref, in place, in the moment space of
// the Gram-Schmidt matrix M of Eq. MatrixMRT (rows rho, e, zeta, j_x, q_x,
// j_y, q_y, p_xx, p_xy):
//   m* = m - Lambda (m - m^eq) + (I - Lambda/2) S_bar,   d* = M^-1 m*
// with m^eq and S_bar = M s of Appendix A.  For the deviations, M (w rho_ref)
// = rho_ref (1, -2, 1, 0, ..., 0) is taken out of the rho, e and zeta rows.
// The rho row is unchanged (m = m^eq, no source) and the momentum rows give
// m_j + F for every rate (m_j - m_j^eq = -F/2), so tau_rho and tau_j drop out.
// The rows of M are orthogonal, so M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12,
// 1/6, 1/12, 1/4, 1/4).
template <class R>
__device__ __forceinline__ void collide_mrt(R d[kQ], R rho, R ux, R uy, R Fx, R Fy,
                                            const Phys<R> &P)
{
    const R dr = (((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7]))) + d[8];
    const R ax = (d[1] + d[2]) + (d[3] + d[4]);             // axis directions
    const R dg = (d[5] + d[6]) + (d[7] + d[8]);             // diagonal directions
    const R e = fma(R(-4), d[0], fma(R(2), dg, -ax));
    const R z = fma(R(4), d[0], fma(R(-2), ax, dg));
    const R jx = ((d[1] - d[3]) + (d[5] - d[6])) + (d[8] - d[7]);
    const R jy = ((d[2] - d[4]) + (d[5] + d[6])) - (d[7] + d[8]);
    const R qx = fma(R(-2), d[1] - d[3], (d[5] - d[7]) + (d[8] - d[6]));
    const R qy = fma(R(-2), d[2] - d[4], (d[5] - d[7]) + (d[6] - d[8]));
    const R pxx = (d[1] + d[3]) - (d[2] + d[4]);
    const R pxy = (d[5] + d[7]) - (d[6] + d[8]);

    const R usq = fma(ux, ux, uy * uy);
    const R uF6 = R(6) * fma(ux, Fx, uy * Fy);
    const R rusq3 = R(3) * rho * usq;
    const R se = P.s_e, sz = P.s_z, sq = P.s_q, sn = P.omega;
    const R es = fma(R(1) - se, e, fma(se, fma(R(-2), dr, rusq3), (R(1) - R(0.5) * se) * uF6));
    const R zs = fma(R(1) - sz, z, fma(sz, dr - rusq3, -(R(1) - R(0.5) * sz) * uF6));
    const R jxs = jx + Fx, jys = jy + Fy;
    const R gq = R(1) - R(0.5) * sq;
    const R qxs = fma(R(1) - sq, qx, -fma(sq * rho, ux, gq * Fx));
    const R qys = fma(R(1) - sq, qy, -fma(sq * rho, uy, gq * Fy));
    const R gn = R(1) - R(0.5) * sn;
    const R pxxs = fma(R(1) - sn, pxx,
                       fma(sn * rho, fma(ux, ux, -uy * uy), gn * R(2) * fma(ux, Fx, -uy * Fy)));
    const R pxys = fma(R(1) - sn, pxy, fma(sn * rho, ux * uy, gn * fma(ux, Fy, uy * Fx)));

    const R r9 = dr * R(1.0 / 9.0);
    const R A1 = fma(es, R(-1.0 / 36.0), fma(zs, R(-1.0 / 18.0), r9));
    const R A2 = fma(es, R(1.0 / 18.0), fma(zs, R(1.0 / 36.0), r9));
    const R X1 = (jxs - qxs) * R(1.0 / 6.0), Y1 = (jys - qys) * R(1.0 / 6.0);
    const R X2 = fma(jxs, R(1.0 / 6.0), qxs * R(1.0 / 12.0));
    const R Y2 = fma(jys, R(1.0 / 6.0), qys * R(1.0 / 12.0));
    const R Pp = pxxs * R(0.25), Qp = pxys * R(0.25);
    d[0] = fma(zs - es, R(1.0 / 9.0), r9);
    d[1] = (A1 + X1) + Pp;
    d[2] = (A1 + Y1) - Pp;
    d[3] = (A1 - X1) + Pp;
    d[4] = (A1 - Y1) - Pp;
    d[5] = (A2 + X2) + (Y2 + Qp);
    d[6] = (A2 - X2) + (Y2 - Qp);
    d[7] = (A2 - X2) - (Y2 - Qp);
    d[8] = (A2 + X2) - (Y2 + Qp);
}

__device__ __forceinline__ double weight(int i)
{
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
}

// Equilibrium (Eq. SEDF) of direction i, FP64.
__device__ __forceinline__ double feq_dir(int i, double rho, double ux, double uy)
{
    const int cx[kQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int cy[kQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const double cu = cx[i] * ux + cy[i] * uy;
    return weight(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy));
}

template <int BX>
__device__ __forceinline__ double warp_or_block_sum(double v, double *lds_red)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    constexpr int W = BX / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds_red[wid] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k)
        s += lds_red[k];
    return s;
}

template <int BX>
__device__ __forceinline__ double warp_or_block_max(double v, double *lds_red)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v = fmax(v, __shfl_xor(v, off, 64));
    constexpr int W = BX / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds_red[wid] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k)
        s = fmax(s, lds_red[k]);
    return s;
}

// psi (own column o, x - 1 in l, x + 1 in r) and rho (own column) of one row.
template <class R>
struct Row {
    R l, o, r, rho;
};

// psi(x + c_i) for the current row C when the walk goes in direction DIR
// (+1: the leading row L is y + 1 and the trailing row T is y - 1; -1: the
// other way round).
template <int DIR, class R>
__device__ __forceinline__ void stencil(const Row<R> &T, const Row<R> &C, const Row<R> &L,
                                        R s[kQ])
{
    const Row<R> &U = DIR > 0 ? L : T;  // row y + 1
    const Row<R> &D = DIR > 0 ? T : L;  // row y - 1
    s[0] = C.o;
    s[1] = C.r;
    s[2] = U.o;
    s[3] = C.l;
    s[4] = D.o;
    s[5] = U.r;
    s[6] = U.l;
    s[7] = D.l;
    s[8] = D.r;
}

// Calls f(integral_constant<int, J>) for J = 0 .. N-1, fully unrolled.
template <class F, int... J>
__device__ __forceinline__ void unroll(F &&f, std::integer_sequence<int, J...>)
{
    (f(std::integral_constant<int, J>{}), ...);
}

// One workgroup walks rows [ys, ye) of its strip in direction DIR, with the
// populations of PF rows beyond the leading row in flight.  K = PF + 2
// population register sets and K psi rows rotate through their roles; the
// loop is unrolled K times so that the rotation is register renaming.
//   row k (0-based within the segment) is output row y0 + k DIR;
//   at iteration k: populations of row k are in set k % K (collided),
//   of row k + 1 in set (k + 1) % K (turned into the leading psi row), and
//   row k + 1 + PF is loaded into set (k + 1 + PF) % K;
//   psi rows k - 1, k, k + 1 are in rows (k) % K, (k + 1) % K, (k + 2) % K.
// The row body is straight-line code: every lane loads (lanes outside the
// strip read a valid column, rows past the segment end are clamped to its
// halo row) and computes; only the stores are masked.  Without branches
// around the loads the compiler's wait counters stay exact, so a prefetch
// really stays in flight while the current row is computed.  Domain
// failures are folded into a per-lane minimum key and published once.
//
// Per-cell mode: the reference R of each lattice row is loaded once (with one
// side neighbour), one row ahead of the populations that need it, and the
// other neighbour comes through a second double-buffered LDS row (a second
// barrier per row).  The triples of R of the segment rows k, k + 1, k + 2
// rotate with the population sets; the lead row k + 1 is reconstructed from
// them when it is turned into psi.
template <int BX, int MODE, int DIR, int PF, int FORCE, int ST, int COLL>
__device__ __forceinline__ void walk(const typename Store<ST>::E *__restrict__ src,
                                     typename Store<ST>::E *__restrict__ dst, const Coeffs &c,
                                     long long t, const Fields &fo, double *__restrict__ rho_snap,
                                     int ys, int ye, int x, const Cols &cols, bool active,
                                     bool interior, typename Store<ST>::R *lds, float *ldsr,
                                     double acc[kDiag], unsigned long long &bad)
{
    using E = typename Store<ST>::E;
    using R = typename Store<ST>::R;
    constexpr bool LOC = Store<ST>::local;
    constexpr int K = PF + 2;
    const Phys<R> P(c);
    const int tx = threadIdx.x;
    const int txm = tx > 0 ? tx - 1 : 0, txp = tx < BX - 1 ? tx + 1 : BX - 1;
    const int nrows = ye - ys;
    const int y0 = DIR > 0 ? ys : ye - 1;
    // wrapped lattice row of segment row k (k in [-1, nrows])
    auto lattice_row = [&](int k) {
        const int r = y0 + k * DIR;
        return r < 0 ? r + c.ny : (r >= c.ny ? r - c.ny : r);
    };
    auto check = [&](bool ok, int r) {
        if (!ok && active) bad = min(bad, domain_key(t, r, x, c.nx));
    };

    R f[K][kQ];
    Row<R> rw[K];
    // per-cell mode: raw R of segment rows (slot = row mod K) and the triples
    RefPair<R> rl[K];
    Tri<R> tr[K];
    const R gref = (R)c.rho_ref;  // the shifted modes' reference density
    const bool first = tx == 0;
    // the left neighbour of every lane but the first comes from the lane on
    // its left; the right neighbour was loaded (the first lane takes it from
    // lane 1)
    auto tri_of = [&](const RefPair<R> &v, float *buf) {
        buf[tx] = (float)v.own;
        __syncthreads();
        return first ? Tri<R>{v.side, v.own, (R)buf[1]} : Tri<R>{(R)buf[txm], v.own, v.side};
    };
    // lattice rows r - 1 and r + 1 of segment row k are segment rows k - DIR and k + DIR
    auto rebuild = [&](R d[kQ], const Tri<R> &prev, const Tri<R> &here, const Tri<R> &next) {
        if (DIR > 0)
            reconstruct<R>(d, prev, here, next);
        else
            reconstruct<R>(d, next, here, prev);
    };

    // prologue: psi of the trailing row (rw[0]) and the current row (rw[1]);
    // populations of segment rows 0 .. PF (clamped to nrows) into sets 0 .. PF;
    // per-cell mode: R of segment rows -2 .. PF + 1 (clamped to nrows + 1)
    {
        R ft[kQ];
        const int rt = lattice_row(-1);
        load_pulled<ST>(src, c, rt, cols, ft);
        load_pulled<ST>(src, c, y0, cols, f[0]);
#pragma unroll
        for (int p = 1; p <= PF; ++p)
            load_pulled<ST>(src, c, lattice_row(p < nrows ? p : nrows), cols, f[p]);
        R reft = gref, ref0 = gref;
        if constexpr (LOC) {
            const RefPair<R> rm2 = load_ref<R>(src, c, lattice_row(-2), cols, first);
            const RefPair<R> rm1 = load_ref<R>(src, c, rt, cols, first);
#pragma unroll
            for (int p = 0; p <= PF + 1; ++p)
                rl[p % K] = load_ref<R>(src, c, lattice_row(p < nrows + 1 ? p : nrows + 1), cols,
                                        first);
            const Tri<R> tm2 = tri_of(rm2, ldsr);
            const Tri<R> tm1 = tri_of(rm1, ldsr + BX);
            tr[0] = tri_of(rl[0], ldsr + 2 * BX);
            tr[1 % K] = tri_of(rl[1 % K], ldsr + 3 * BX);
            rebuild(ft, tm2, tm1, tr[0]);
            rebuild(f[0], tm1, tr[0], tr[1 % K]);
            reft = tm1.o;
            ref0 = tr[0].o;
            __syncthreads();  // ldsr is rewritten by the first row
        }
        check(rho_psi<FORCE, R>(ft, reft, P, rw[0].rho, rw[0].o), rt);
        check(rho_psi<FORCE, R>(f[0], ref0, P, rw[1].rho, rw[1].o), y0);
        lds[tx] = rw[0].o;
        lds[BX + tx] = rw[1].o;
        __syncthreads();
        rw[0].l = lds[txm];
        rw[0].r = lds[txp];
        rw[1].l = lds[BX + txm];
        rw[1].r = lds[BX + txp];
        __syncthreads();
    }

    auto body = [&](auto Jc, int k) {
        constexpr int J = decltype(Jc)::value;      // k % K
        constexpr int cur = J % K, lead = (J + 1) % K, fetch = (J + 1 + PF) % K;
        const Row<R> &T = rw[J % K];
        const Row<R> &C = rw[(J + 1) % K];
        Row<R> &L = rw[(J + 2) % K];
        const int y = y0 + k * DIR;
        {
            const int kf = k + 1 + PF;
            load_pulled<ST>(src, c, lattice_row(kf < nrows ? kf : nrows), cols, f[fetch]);
        }
        R ref_cur = gref, ref_lead = gref;
        if constexpr (LOC) {
            // R of segment row k + 2 + PF into slot J (row k is done with it);
            // the triple of row k + 2 completes the lead row k + 1
            const int kr = k + 2 + PF;
            const RefPair<R> nr =
                load_ref<R>(src, c, lattice_row(kr < nrows + 1 ? kr : nrows + 1), cols, first);
            tr[(J + 2) % K] = tri_of(rl[(J + 2) % K], ldsr + (k & 1) * BX);
            rl[J % K] = nr;
            rebuild(f[lead], tr[J % K], tr[(J + 1) % K], tr[(J + 2) % K]);
            ref_cur = tr[J % K].o;
            ref_lead = tr[(J + 1) % K].o;
        }
        check(rho_psi<FORCE, R>(f[lead], ref_lead, P, L.rho, L.o), lattice_row(k + 1));
        R *buf = lds + (k & 1) * BX;
        buf[tx] = L.o;
        __syncthreads();
        L.l = buf[txm];
        L.r = buf[txp];
        R Fx = R(0), Fy = R(0);
        if (FORCE) {
            R s[kQ];
            stencil<DIR, R>(T, C, L, s);
            force<R>(s, P, Fx, Fy);
        }
        R ux, uy;
        velocity<R>(f[cur], C.rho, Fx, Fy, ux, uy);
        const size_t row = (size_t)y * c.nx;
        if (MODE == kStep) {
            if constexpr (COLL == LBM_COLL_MRT)
                collide_mrt<R>(f[cur], C.rho, ux, uy, Fx, Fy, P);
            else
                collide<R>(f[cur], ref_cur, C.rho, ux, uy, Fx, Fy, P);
            if (interior) {
                const size_t prow = (size_t)y * c.pitch;
                if constexpr (Store<ST>::local) {
                    // per-cell reference: the new R = sum_i f*_i = ref + s with
                    // s = sum_i d*_i, X_i = round(f*_i - w_i R) = round(d*_i - w_i s),
                    // then R corrected by the rounding errors so that the cell's
                    // nine X_i + w_i R keep its mass
                    const R *g = f[cur];
                    const R sd =
                        (((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7]))) +
                        g[8];
                    R err = R(0);
#pragma unroll
                    for (int i = 0; i < kQ; ++i) {
                        const R w = i == 0 ? R(4.0 / 9.0) : (i < 5 ? R(1.0 / 9.0) : R(1.0 / 36.0));
                        const R dev = fma(-w, sd, g[i]);
                        const E X = (E)dev;
                        err += dev - (R)X;
                        __builtin_nontemporal_store(
                            X, (E *)((char *)(dst + i * c.plane + prow) + cols.o));
                    }
                    float *rrow = (float *)((char *)dst + c.r_off) + (size_t)y * c.r_pitch;
                    __builtin_nontemporal_store((float)(ref_cur + (sd + err)),
                                                (float *)((char *)rrow + 2 * cols.o));
                } else {
#pragma unroll
                    for (int i = 0; i < kQ; ++i)
                        __builtin_nontemporal_store(
                            (E)f[cur][i], (E *)((char *)(dst + i * c.plane + prow) + cols.o));
                }
            }
        } else if (MODE == kMoments) {
            if (interior) {
                const size_t cell = row + x;
                if (fo.rho) fo.rho[cell] = (double)C.rho;
                if (fo.ux) fo.ux[cell] = (double)ux;
                if (fo.uy) fo.uy[cell] = (double)uy;
                if (fo.Fx) fo.Fx[cell] = (double)Fx;
                if (fo.Fy) fo.Fy[cell] = (double)Fy;
                if (fo.psi) fo.psi[cell] = (double)C.o;
            }
        } else {
            if (interior) {
                const size_t cell = row + x;
                const double r64 = (double)C.rho, ux64 = (double)ux, uy64 = (double)uy;
                const double prev = rho_snap[cell];
                rho_snap[cell] = r64;
                acc[0] += r64;
                acc[1] += r64 * ux64;
                acc[2] += r64 * uy64;
                acc[3] += fabs(r64 - prev);
                acc[4] += fabs(r64);
                acc[5] = fmax(acc[5], sqrt(ux64 * ux64 + uy64 * uy64));
            }
        }
    };

    int k = 0;
    for (; k + K <= nrows; k += K)
        unroll([&](auto J) { body(J, k + decltype(J)::value); },
               std::make_integer_sequence<int, K>{});
    unroll([&](auto J) {
        if (k + decltype(J)::value < nrows) body(J, k + decltype(J)::value);
    }, std::make_integer_sequence<int, K - 1>{});
}

// One tile of a sweep: strip `strip` of row band `seg` of one lattice.
template <int BX, int MODE, int PF, int FORCE, int ST, int COLL>
__device__ __forceinline__ void sweep_tile(const void *__restrict__ src_v, void *__restrict__ dst_v,
                                           const Coeffs &c, const Tiles &tl, int tile,
                                           long long t, unsigned long long *__restrict__ err,
                                           const Fields &fo, double *__restrict__ rho_snap,
                                           double *__restrict__ partials)
{
    using E = typename Store<ST>::E;
    using R = typename Store<ST>::R;
    const E *src = (const E *)src_v;
    E *dst = (E *)dst_v;
    __shared__ R lds[2 * BX];
    __shared__ float ldsr[Store<ST>::local ? 4 * BX : 1];
    const int seg = tile / tl.nstrips;
    const int strip = tile - seg * tl.nstrips;
    const int xs = strip * tl.width;
    const int xe = min(c.nx, xs + tl.width);
    const int ys = (int)((long long)seg * c.ny / tl.nseg);
    const int ye = (int)((long long)(seg + 1) * c.ny / tl.nseg);

    const int tx = threadIdx.x;
    const int width = xe - xs;                 // interior columns, <= BX - 2
    const bool active = tx <= width + 1;
    const bool interior = tx >= 1 && tx <= width;
    int x = xs - 1 + (active ? tx : 1);
    x = wrap_hi(wrap_lo(x, c.nx), c.nx);
    const int xm = wrap_lo(x - 1, c.nx), xp = wrap_hi(x + 1, c.nx);
    constexpr uint32_t es = sizeof(E);
    const Cols cols{(uint32_t)x * es, (uint32_t)xm * es, (uint32_t)xp * es};

    double acc[kDiag] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    unsigned long long bad = ~0ull;
    if (seg & 1)
        walk<BX, MODE, -1, PF, FORCE, ST, COLL>(src, dst, c, t, fo, rho_snap, ys, ye, x, cols, active,
                                          interior, lds, ldsr, acc, bad);
    else
        walk<BX, MODE, +1, PF, FORCE, ST, COLL>(src, dst, c, t, fo, rho_snap, ys, ye, x, cols, active,
                                          interior, lds, ldsr, acc, bad);
    if (bad != ~0ull) atomicMin(err, bad);

    if (MODE == kDiagnostics) {
        __shared__ double red[BX / 64];
        double out[kDiag];
#pragma unroll
        for (int j = 0; j < kDiag - 1; ++j)
            out[j] = warp_or_block_sum<BX>(acc[j], red);
        out[kDiag - 1] = warp_or_block_max<BX>(acc[kDiag - 1], red);
        if (tx == 0) {
#pragma unroll
            for (int j = 0; j < kDiag; ++j)
                partials[(size_t)tile * kDiag + j] = out[j];
        }
    }
}

// Workgroups are dealt to the 8 XCDs of the chip round-robin (workgroup b
// runs on XCD b mod 8), and each XCD has an L2 of its own.  Tile of workgroup
// b among n tiles numbered row band by row band: XCD k takes the contiguous
// run of tiles [start(k), start(k + 1)), so the workgroups that share a
// segment's halo rows or a strip's halo columns run on the same XCD, at about
// the same time, and re-read them from its L2.  A bijection of [0, n) for
// every n.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int xcd = b & 7, j = b >> 3, base = n >> 3, rem = n & 7;
    return xcd * base + min(xcd, rem) + j;
}

// Waves per SIMD the compiler must leave room for: the per-cell mode with the
// BGK collision holds one register more than four waves allow without the
// bound (with it, 128 and no spills; the MRT variant would spill, so it runs
// at three waves).
template <int ST, int COLL>
constexpr int kMinWaves = (Store<ST>::local && COLL == LBM_COLL_BGK) ? 4 : 1;

// One sweep over one lattice.
template <int BX, int MODE, int PF, int FORCE, int ST, int COLL>
__global__ __launch_bounds__(BX, (kMinWaves<ST, COLL>)) void sweep_kernel(const void *__restrict__ src,
                                                   void *__restrict__ dst, Coeffs c, Tiles tl,
                                                   long long t,
                                                   unsigned long long *__restrict__ err,
                                                   Fields fo, double *__restrict__ rho_snap,
                                                   double *__restrict__ partials)
{
    sweep_tile<BX, MODE, PF, FORCE, ST, COLL>(src, dst, c, tl, xcd_tile(blockIdx.x, tl.ntiles),
                                              t, err, fo, rho_snap, partials);
}

// One lattice of a batch, as the batched step kernel sees it.
struct BatchEntry {
    Coeffs c;
    Tiles tl, tl2;            // tiles of a single step and of the two-step pass
    const void *buf[2];       // population buffers; the first batched launch reads buf[0]
    unsigned long long *err;  // the lattice's sticky error word
    long long t0;             // the lattice's step count before the batched steps
    int tile0, tile0_2;       // its first tile in the single-step / two-step batch grid
};

// Lattice of batch tile b: the last entry whose first tile (member F) is <= b
// (binary search over the table, uniform per workgroup).
template <int BatchEntry::*F>
__device__ __forceinline__ const BatchEntry &batch_entry(const BatchEntry *__restrict__ table,
                                                         int nlat, int b)
{
    int lo = 0, hi = nlat - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (table[mid].*F <= b) lo = mid;
        else hi = mid - 1;
    }
    return table[lo];
}

// One time step of every lattice of a batch: workgroup b takes batch tile
// xcd_tile(b) and runs tile b - tile0 of its lattice.  The steps and the
// launches since the table was written are read from d_ctr[0] and d_ctr[1]
// (so that a captured graph replays correctly): the first gives the time,
// the parity of the second the source buffer.
template <int BX, int PF, int FORCE, int ST, int COLL>
__global__ __launch_bounds__(BX, (kMinWaves<ST, COLL>)) void batch_step_kernel(const BatchEntry *__restrict__ table,
                                                        int nlat,
                                                        const long long *__restrict__ d_ctr)
{
    const long long steps = d_ctr[0];
    const int parity = (int)(d_ctr[1] & 1);
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const BatchEntry &e = batch_entry<&BatchEntry::tile0>(table, nlat, b);
    sweep_tile<BX, kStep, PF, FORCE, ST, COLL>(e.buf[parity], (void *)e.buf[parity ^ 1], e.c,
                                               e.tl, b - e.tile0, e.t0 + steps, e.err, Fields{},
                                               nullptr, nullptr);
}

// Two time steps in one pass, t -> t + 2: the populations are read once and
// written once for two updates.  Step A (time t) is the single-step update on
// the loaded rows; step B (time t + 1) pulls A's post-collision values from
// LDS.  The update of a cell depends on the cells within two of it, so B's
// output strip is narrower than A's by three columns on each side (A's force
// needs psi one column beyond, B pulls one column beyond A's valid results,
// and B's force needs psi one column beyond that), and B's output rows
// [0, n) need A's rows [-2, n + 1] and psi of A's rows [-3, n + 2].  Both
// steps call the same routines as the single-step walk, in the same order, on
// the same values (A's results rounded to the storage type, as a single step
// stores them), so the result is bitwise that of two single steps.
//
// The walk runs m = 0 .. n + 5; iteration m
//   prefetches A's populations of row m - 2,
//   turns A's row m - 3 into rho and psi (psi to LDS; barrier 1),
//   collides A's row m - 4 and hands it to B (barrier 2),
//   pulls B's row m - 5 and turns it into rho and psi (psi to LDS; barrier 3),
//   pulls B's row m - 6 again, collides it and stores it.
// psi rows live in LDS rings of three rows (slot = iteration mod 3); the
// force reads its 3 x 3 window there.  Of A's post-collision values only the
// populations that B pulls from a neighbouring lane go through LDS, each kept
// as long as B reads it: 7 and 8 (pulled from row r + 1) two iterations, 1 and
// 3 (row r) three, 5 and 6 (row r - 1) four.  Populations 0, 2 and 4 come
// from the own lane and stay in registers.  Register sets rotate with period 6
// (the loop is unrolled six times).
template <class R, int BX, bool LOC>
struct Pass2Lds {
    R psi_a[3][BX], psi_b[3][BX];  // psi of A's and B's rows
    R p78[2][2][BX];               // populations 7, 8 of A's rows
    R p13[3][2][BX];               // populations 1, 3
    R p56[4][2][BX];               // populations 5, 6
    // per-cell mode: the reference R of A's input rows (exchanged for the
    // neighbours' values) and the new R of A's output rows (B reads it for
    // rows r - 1, r, r + 1, so four rows live at once)
    float r_in[LOC ? 2 : 1][BX], r_out[LOC ? 4 : 1][BX];
};

template <int BX, int PF, int FORCE, int ST, int COLL>
__device__ __forceinline__ void walk2(const typename Store<ST>::E *__restrict__ src,
                                      typename Store<ST>::E *__restrict__ dst, const Coeffs &c,
                                      long long t, int ys, int n, int x, const Cols &cols,
                                      bool active, bool valid_b, bool interior,
                                      Pass2Lds<typename Store<ST>::R, BX, Store<ST>::local> &L,
                                      unsigned long long &bad)
{
    using E = typename Store<ST>::E;
    using R = typename Store<ST>::R;
    constexpr bool LOC = Store<ST>::local;
    static_assert(PF == 1, "the period-6 rotation assumes one row of prefetch");
    constexpr int K = PF + 2;
    const Phys<R> P(c);
    const R gref = (R)c.rho_ref;
    const int tx = threadIdx.x;
    const int txm = tx > 0 ? tx - 1 : 0, txp = tx < BX - 1 ? tx + 1 : BX - 1;
    auto lrow = [&](int s) {
        const int r = (ys + s) % c.ny;
        return r < 0 ? r + c.ny : r;
    };
    auto check = [&](bool ok, long long step, int s) {
        if (!ok) bad = min(bad, domain_key(step, lrow(s), x, c.nx));
    };
    // psi window row of slot s of a ring
    auto psi_row = [&](const R(*ring)[BX], int s) {
        return Row<R>{ring[s][txm], ring[s][tx], ring[s][txp], R(0)};
    };

    R fa[K][kQ];
    R rho_a[2], rho_b[2];   // rho of the last two psi rows of each step
    R h0[3], h2[6], h4[2];  // populations 0, 2, 4 of A's last post-collision rows
    // per-cell mode: R triples of A's input rows (slot = (row + 1) mod 3), R
    // of A's rows before their collision, R of the next rows in flight
    Tri<R> ta[3];
    R ra[2];
    RefPair<R> rl[2];
    const bool first = tx == 0;
    // R at x - 1, x, x + 1 from a lane's own and side values and an LDS row
    auto tri_from = [&](const RefPair<R> &v, const float *buf) {
        return first ? Tri<R>{v.side, v.own, (R)buf[1]} : Tri<R>{(R)buf[txm], v.own, v.side};
    };
    auto tri_lds = [&](const float *buf) {
        return Tri<R>{(R)buf[txm], (R)buf[tx], (R)buf[txp]};
    };
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            fa[k][i] = R(0);
    }
    rho_a[0] = rho_a[1] = rho_b[0] = rho_b[1] = R(0);
#pragma unroll
    for (int k = 0; k < 6; ++k)
        h2[k] = R(0);
    h0[0] = h0[1] = h0[2] = h4[0] = h4[1] = R(0);
    ra[0] = ra[1] = R(0);
    // prologue: A's populations of rows -3 .. -4 + PF
#pragma unroll
    for (int p = 0; p < PF; ++p)
        load_pulled<ST>(src, c, lrow(-3 + p), cols, fa[(1 + p) % K]);
    if constexpr (LOC) {
        // R triples of rows -4, -3, -2 (slots 0, 1, 2), exchanged through
        // three rows of r_out behind one barrier (r_out is first written two
        // iterations later, after two more barriers); R of row -1 in flight
        const RefPair<R> q4 = load_ref<R>(src, c, lrow(-4), cols, first);
        const RefPair<R> q3 = load_ref<R>(src, c, lrow(-3), cols, first);
        const RefPair<R> q2 = load_ref<R>(src, c, lrow(-2), cols, first);
        rl[1] = load_ref<R>(src, c, lrow(-1), cols, first);
        rl[0] = rl[1];
        L.r_out[0][tx] = (float)q4.own;
        L.r_out[1][tx] = (float)q3.own;
        L.r_out[2][tx] = (float)q2.own;
        __syncthreads();
        ta[0] = tri_from(q4, L.r_out[0]);
        ta[1] = tri_from(q3, L.r_out[1]);
        ta[2] = tri_from(q2, L.r_out[2]);
    }

    // gates: the first iterations skip the work on rows no output needs (A's
    // collision of rows -4, -3, B's psi of rows -5 .. -2, B's collision of
    // rows -6 .. -1); FIRST marks an iteration of the peeled first six
    auto body = [&](auto Jc, auto firstc, int m) {
        constexpr int J = decltype(Jc)::value;  // m % 6
        constexpr bool FIRST = decltype(firstc)::value;
        constexpr bool DO_A = !FIRST || J >= 2, DO_BPSI = !FIRST || J >= 4, DO_BCOL = !FIRST;
        constexpr int a_cur = J % K, a_lead = (J + 1) % K, a_fetch = (J + 1 + PF) % K;
        {
            const int s = m - 3 + PF;
            load_pulled<ST>(src, c, lrow(s < n + 2 ? s : n + 2), cols, fa[a_fetch]);
        }
        // step A: rho and psi of row m - 3 (always one of A's rows -3 .. n + 2);
        // per-cell mode: its deviations are rebuilt from R of rows m - 4 ..
        // m - 2 first, and R of row m - 1 is exchanged through the same barrier
        {
            R ref_lead = gref;
            if constexpr (LOC) {
                reconstruct<R>(fa[a_lead], ta[J % 3], ta[(J + 1) % 3], ta[(J + 2) % 3]);
                ref_lead = ta[(J + 1) % 3].o;
                ra[J % 2] = ref_lead;
                L.r_in[J % 2][tx] = (float)rl[(J + 1) % 2].own;
                rl[J % 2] = load_ref<R>(src, c, lrow(m), cols, first);
            }
            R psi;
            const bool ok = rho_psi<FORCE, R>(fa[a_lead], ref_lead, P, rho_a[J % 2], psi);
            if (active) check(ok, t, m - 3);
            L.psi_a[J % 3][tx] = psi;
            __syncthreads();
            if constexpr (LOC) ta[J % 3] = tri_from(rl[(J + 1) % 2], L.r_in[J % 2]);
        }
        // step A: collision of row m - 4; B's share of it to LDS and registers
        if constexpr (DO_A) {
            R Fx = R(0), Fy = R(0);
            if (FORCE) {
                const Row<R> T = psi_row(L.psi_a, (J + 1) % 3);
                const Row<R> C = psi_row(L.psi_a, (J + 2) % 3);
                const Row<R> U = psi_row(L.psi_a, J % 3);
                R sv[kQ];
                stencil<+1, R>(T, C, U, sv);
                force<R>(sv, P, Fx, Fy);
            }
            R *g = fa[a_cur];
            const R rho = rho_a[(J + 1) % 2];
            const R ref_cur = LOC ? ra[(J + 1) % 2] : gref;
            R ux, uy;
            velocity<R>(g, rho, Fx, Fy, ux, uy);
            if constexpr (COLL == LBM_COLL_MRT)
                collide_mrt<R>(g, rho, ux, uy, Fx, Fy, P);
            else
                collide<R>(g, ref_cur, rho, ux, uy, Fx, Fy, P);
            // encoded as a single step stores them: rounded to the storage
            // type; per-cell mode: X_i = round(d*_i - w_i s) with s the sum of
            // the d*_i, and the new R = ref + (s + rounding errors)
            if constexpr (LOC) {
                const R sd =
                    (((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7]))) + g[8];
                R err = R(0);
#pragma unroll
                for (int i = 0; i < kQ; ++i) {
                    const R w = i == 0 ? R(4.0 / 9.0) : (i < 5 ? R(1.0 / 9.0) : R(1.0 / 36.0));
                    const R dev = fma(-w, sd, g[i]);
                    const E X = (E)dev;
                    err += dev - (R)X;
                    g[i] = (R)X;
                }
                L.r_out[m & 3][tx] = (float)(ref_cur + (sd + err));
            }
            auto rd = [&](int i) { return LOC ? g[i] : (R)(E)g[i]; };
            h0[J % 3] = rd(0);
            h2[J] = rd(2);
            h4[J % 2] = rd(4);
            L.p13[J % 3][0][tx] = rd(1);
            L.p13[J % 3][1][tx] = rd(3);
            L.p56[m & 3][0][tx] = rd(5);
            L.p56[m & 3][1][tx] = rd(6);
            L.p78[J % 2][0][tx] = rd(7);
            L.p78[J % 2][1][tx] = rd(8);
        }
        __syncthreads();
        // B's pulled populations of row m - 5 - back (back = 0: the row turned
        // into psi now, back = 1: the row collided now); A's row q was written
        // at iteration q + 4
        auto pull_b = [&](auto backc, R g[kQ]) {
            constexpr int b = decltype(backc)::value;
            constexpr int s2 = (J + 2 - b) % 2, s3r = (J + 5 - b) % 3, s6 = (J + 10 - b) % 6;
            const int s4 = (m + 2 - b) & 3;
            // row r + 1 (written at m - b), row r (m - 1 - b), row r - 1 (m - 2 - b)
            g[4] = h4[s2];
            g[7] = L.p78[s2][0][txp];
            g[8] = L.p78[s2][1][txm];
            g[0] = h0[s3r];
            g[1] = L.p13[s3r][0][txm];
            g[3] = L.p13[s3r][1][txp];
            g[2] = h2[s6];
            g[5] = L.p56[s4][0][txm];
            g[6] = L.p56[s4][1][txp];
        };
        // step B: rho and psi of row m - 5
        if constexpr (DO_BPSI) {
            R g[kQ];
            pull_b(std::integral_constant<int, 0>{}, g);
            R ref_b = gref;
            if constexpr (LOC) {
                // rows r + 1, r, r - 1 were handed over at m, m - 1, m - 2
                const Tri<R> C = tri_lds(L.r_out[(m + 3) & 3]);
                reconstruct<R>(g, tri_lds(L.r_out[(m + 2) & 3]), C, tri_lds(L.r_out[m & 3]));
                ref_b = C.o;
            }
            R psi;
            const bool ok = rho_psi<FORCE, R>(g, ref_b, P, rho_b[J % 2], psi);
            if (valid_b && m - 5 >= -1) check(ok, t + 1, m - 5);
            L.psi_b[J % 3][tx] = psi;
        }
        __syncthreads();
        // step B: collision of row m - 6 and its store
        if constexpr (DO_BCOL) {
            R g[kQ];
            pull_b(std::integral_constant<int, 1>{}, g);
            R ref_cur = gref;
            if constexpr (LOC) {
                // rows r + 1, r, r - 1 were handed over at m - 1, m - 2, m - 3
                const Tri<R> C = tri_lds(L.r_out[(m + 2) & 3]);
                reconstruct<R>(g, tri_lds(L.r_out[(m + 1) & 3]), C, tri_lds(L.r_out[(m + 3) & 3]));
                ref_cur = C.o;
            }
            R Fx = R(0), Fy = R(0);
            if (FORCE) {
                const Row<R> T = psi_row(L.psi_b, (J + 1) % 3);
                const Row<R> C = psi_row(L.psi_b, (J + 2) % 3);
                const Row<R> U = psi_row(L.psi_b, J % 3);
                R sv[kQ];
                stencil<+1, R>(T, C, U, sv);
                force<R>(sv, P, Fx, Fy);
            }
            const R rho = rho_b[(J + 1) % 2];
            R ux, uy;
            velocity<R>(g, rho, Fx, Fy, ux, uy);
            if constexpr (COLL == LBM_COLL_MRT)
                collide_mrt<R>(g, rho, ux, uy, Fx, Fy, P);
            else
                collide<R>(g, ref_cur, rho, ux, uy, Fx, Fy, P);
            const int sb = m - 6;
            if (interior && sb >= 0 && sb < n) {
                const int yb = lrow(sb);
                const size_t prow = (size_t)yb * c.pitch;
                if constexpr (LOC) {
                    // as the single-step store of the per-cell mode
                    const R sd =
                        (((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7]))) +
                        g[8];
                    R err = R(0);
#pragma unroll
                    for (int i = 0; i < kQ; ++i) {
                        const R w = i == 0 ? R(4.0 / 9.0) : (i < 5 ? R(1.0 / 9.0) : R(1.0 / 36.0));
                        const R dev = fma(-w, sd, g[i]);
                        const E X = (E)dev;
                        err += dev - (R)X;
                        __builtin_nontemporal_store(
                            X, (E *)((char *)(dst + i * c.plane + prow) + cols.o));
                    }
                    float *rrow = (float *)((char *)dst + c.r_off) + (size_t)yb * c.r_pitch;
                    __builtin_nontemporal_store((float)(ref_cur + (sd + err)),
                                                (float *)((char *)rrow + 2 * cols.o));
                } else {
#pragma unroll
                    for (int i = 0; i < kQ; ++i)
                        __builtin_nontemporal_store(
                            (E)g[i], (E *)((char *)(dst + i * c.plane + prow) + cols.o));
                }
            }
        }
    };

    constexpr int U = 6;
    const int total = n + 6;  // >= 7
    using First = std::true_type;
    using Rest = std::false_type;
    unroll([&](auto J) { body(J, First{}, decltype(J)::value); },
           std::make_integer_sequence<int, U>{});
    int m = U;
    for (; m + U <= total; m += U)
        unroll([&](auto J) { body(J, Rest{}, m + decltype(J)::value); },
               std::make_integer_sequence<int, U>{});
    unroll([&](auto J) {
        if (m + decltype(J)::value < total) body(J, Rest{}, m + decltype(J)::value);
    }, std::make_integer_sequence<int, U - 1>{});
}

// Halo columns of the two-step pass on each side of its output strip.
constexpr int kHalo2 = 3;

// Waves per SIMD the two-step pass is compiled for.  FP64 runs at two (173
// VGPRs with BGK; bounding it to three waves spilled 8 registers and measured
// 2-4% slower); the FP32-arithmetic modes fit four.
template <int ST, int COLL>
constexpr int kWaves2 = ST == LBM_STORE_F64 ? 2 : 4;

// One tile of the two-step pass: output strip `strip` of row band `seg`.
template <int BX, int PF, int FORCE, int ST, int COLL>
__device__ __forceinline__ void sweep2_tile(const void *__restrict__ src_v,
                                            void *__restrict__ dst_v, const Coeffs &c,
                                            const Tiles &tl, int tile, long long t,
                                            unsigned long long *__restrict__ err)
{
    using E = typename Store<ST>::E;
    using R = typename Store<ST>::R;
    __shared__ Pass2Lds<R, BX, Store<ST>::local> lds;
    const int seg = tile / tl.nstrips;
    const int strip = tile - seg * tl.nstrips;
    const int xs = strip * tl.width;
    const int xe = min(c.nx, xs + tl.width);
    const int ys = (int)((long long)seg * c.ny / tl.nseg);
    const int ye = (int)((long long)(seg + 1) * c.ny / tl.nseg);
    const int tx = threadIdx.x;
    const int width = xe - xs;  // output columns, <= BX - 2 kHalo2
    const bool active = tx < width + 2 * kHalo2;
    const bool valid_b = tx >= kHalo2 - 1 && tx <= width + kHalo2;
    const bool interior = tx >= kHalo2 && tx < width + kHalo2;
    int x = (xs - kHalo2 + (active ? tx : kHalo2)) % c.nx;
    x = x < 0 ? x + c.nx : x;
    const int xm = wrap_lo(x - 1, c.nx), xp = wrap_hi(x + 1, c.nx);
    constexpr uint32_t es = sizeof(E);
    const Cols cols{(uint32_t)x * es, (uint32_t)xm * es, (uint32_t)xp * es};
    unsigned long long bad = ~0ull;
    walk2<BX, PF, FORCE, ST, COLL>((const E *)src_v, (E *)dst_v, c, t, ys, ye - ys, x, cols, active,
                                   valid_b, interior, lds, bad);
    if (bad != ~0ull) atomicMin(err, bad);
}

// The two-step pass over one lattice.
template <int BX, int PF, int FORCE, int ST, int COLL>
__global__ __launch_bounds__(BX) __attribute__((amdgpu_waves_per_eu(kWaves2<ST, COLL>)))
void sweep2_kernel(const void *__restrict__ src, void *__restrict__ dst, Coeffs c, Tiles tl,
                   long long t, unsigned long long *__restrict__ err)
{
    sweep2_tile<BX, PF, FORCE, ST, COLL>(src, dst, c, tl, xcd_tile(blockIdx.x, tl.ntiles), t, err);
}

// The two-step pass over every lattice of a batch (tiles and counters as in
// batch_step_kernel; a launch advances two steps and swaps the buffers once).
template <int BX, int PF, int FORCE, int ST, int COLL>
__global__ __launch_bounds__(BX) __attribute__((amdgpu_waves_per_eu(kWaves2<ST, COLL>)))
void batch2_kernel(const BatchEntry *__restrict__ table, int nlat,
                   const long long *__restrict__ d_ctr)
{
    const long long steps = d_ctr[0];
    const int parity = (int)(d_ctr[1] & 1);
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const BatchEntry &e = batch_entry<&BatchEntry::tile0_2>(table, nlat, b);
    sweep2_tile<BX, PF, FORCE, ST, COLL>(e.buf[parity], (void *)e.buf[parity ^ 1], e.c, e.tl2,
                                         b - e.tile0_2, e.t0 + steps, e.err);
}

// Batch counters: p[0] steps, p[1] launches since the table was written.
__global__ void bump_counter(long long *p, long long steps)
{
    p[0] += steps;
    p[1] += 1;
}
__global__ void clear_counters(long long *p)
{
    p[0] = 0;
    p[1] = 0;
}

// Second stage of the diagnostics: one workgroup sums the per-tile partials
// in a fixed order.
__global__ __launch_bounds__(256) void reduce_partials(const double *__restrict__ partials,
                                                        int ntiles, double *__restrict__ out)
{
    __shared__ double red[4];
    double acc[kDiag] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < ntiles; k += 256) {
#pragma unroll
        for (int j = 0; j < kDiag - 1; ++j)
            acc[j] += partials[(size_t)k * kDiag + j];
        acc[kDiag - 1] = fmax(acc[kDiag - 1], partials[(size_t)k * kDiag + kDiag - 1]);
    }
    double res[kDiag];
#pragma unroll
    for (int j = 0; j < kDiag - 1; ++j)
        res[j] = warp_or_block_sum<256>(acc[j], red);
    res[kDiag - 1] = warp_or_block_max<256>(acc[kDiag - 1], red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < kDiag; ++j)
            out[j] = res[j];
    }
}

// The nine FP64 values v_i that cell (x, y) sends (v_i reaches x + c_i) into
// pull storage: the deviation from w_i rho_ref rounded once, or in the
// per-cell mode R = sum_i v_i, X_i = round(v_i - w_i R) and R corrected by
// the rounding errors, rounded to FP32.
template <int ST>
__device__ __forceinline__ void store_cell(void *__restrict__ X_v, const Coeffs &c, int x, int y,
                                           const double v[kQ])
{
    using E = typename Store<ST>::E;
    E *X = (E *)X_v;
    if constexpr (Store<ST>::local) {
        double R = 0.0;
#pragma unroll
        for (int i = 0; i < kQ; ++i)
            R += v[i];
        double err = 0.0;
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const double dev = v[i] - weight(i) * R;
            const E q = (E)dev;
            err += dev - (double)q;
            X[i * c.plane + (size_t)y * c.pitch + x] = q;
        }
        float *rb = (float *)((char *)X_v + c.r_off);
        rb[(size_t)y * c.r_pitch + x] = (float)(R + err);
    } else {
#pragma unroll
        for (int i = 0; i < kQ; ++i)
            X[i * c.plane + (size_t)y * c.pitch + x] = (E)(v[i] - weight(i) * c.rho_ref);
    }
}

// Initial state f(0) = f^eq(rho0, u0) in pull storage: cell z sends f_i^eq at
// z + c_i.
template <int ST>
__global__ __launch_bounds__(256) void init_kernel(void *__restrict__ X_v, Coeffs c,
                                                    const double *__restrict__ rho0,
                                                    const double *__restrict__ ux0,
                                                    const double *__restrict__ uy0)
{
    const size_t n = (size_t)c.nx * c.ny;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int x = (int)(k % c.nx), y = (int)(k / c.nx);
    const int cx[kQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int cy[kQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    double v[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const int xx = wrap_hi(wrap_lo(x + cx[i], c.nx), c.nx);
        const int yy = wrap_hi(wrap_lo(y + cy[i], c.ny), c.ny);
        const size_t s = (size_t)yy * c.nx + xx;
        v[i] = feq_dir(i, rho0[s], ux0 ? ux0[s] : 0.0, uy0 ? uy0[s] : 0.0);
    }
    store_cell<ST>(X_v, c, x, y, v);
}

// Canonical f(t) <-> pull storage.  to_canonical: f_i(x) = w_i rho_ref +
// X_i(x - c_i) (w_i R(x - c_i) + X_i(x - c_i) in the per-cell mode);
// otherwise cell z stores the values f_i(z + c_i) it sends (store_cell).
// Canonical arrays are dense FP64 [9][ny][nx]; the storage has row pitch
// c.pitch and plane stride c.plane.
template <int ST>
__global__ __launch_bounds__(256) void permute_kernel(const void *__restrict__ in_v,
                                                       void *__restrict__ out_v, Coeffs c,
                                                       int to_canonical)
{
    using E = typename Store<ST>::E;
    const size_t n = (size_t)c.nx * c.ny;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int x = (int)(k % c.nx), y = (int)(k / c.nx);
    const int cx[kQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int cy[kQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    if (to_canonical) {
        const E *in = (const E *)in_v;
        double *out = (double *)out_v;
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const int xx = wrap_hi(wrap_lo(x - cx[i], c.nx), c.nx);
            const int yy = wrap_hi(wrap_lo(y - cy[i], c.ny), c.ny);
            const double X = (double)in[i * c.plane + (size_t)yy * c.pitch + xx];
            if constexpr (Store<ST>::local) {
                const float *rb = (const float *)((const char *)in_v + c.r_off);
                out[i * n + k] = X + weight(i) * (double)rb[(size_t)yy * c.r_pitch + xx];
            } else {
                out[i * n + k] = weight(i) * c.rho_ref + X;
            }
        }
    } else {
        const double *in = (const double *)in_v;
        double v[kQ];
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const int xx = wrap_hi(wrap_lo(x + cx[i], c.nx), c.nx);
            const int yy = wrap_hi(wrap_lo(y + cy[i], c.ny), c.ny);
            v[i] = in[i * n + (size_t)yy * c.nx + xx];
        }
        store_cell<ST>(out_v, c, x, y, v);
    }
}

__global__ void fill_u64(unsigned long long *p, unsigned long long v) { *p = v; }

__global__ void copy_plane(const double *__restrict__ a, double *__restrict__ b, size_t n)
{
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) b[k] = a[k];
}

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct lbm_handle {
    lbm_params p;
    Coeffs c;
    hipStream_t stream;
    void *cur, *nxt;         // population buffers (pull storage)
    double *rho_snap;        // density snapshot for Eq. SSC
    double *partials;        // per-tile diagnostics
    double *diag_out;        // kDiag doubles
    unsigned long long *err; // sticky domain-error key
    int64_t t;
    int bx, seg_rows;
    Tiles tiles;
    int fuse;                // time steps per pass of the step kernel (1 or 2)
    int cus;                 // compute units of the device (default shapes)
    int bx2, seg_rows2;      // launch shape of the two-step pass
    Tiles tiles2;
    lbm_status sticky;
    std::string last_error;
};

struct lbm_batch {
    int capacity;
    hipStream_t stream;
    BatchEntry *d_table;
    long long *d_ctr;         // steps and launches since the table was written
    std::vector<lbm_handle *> members;
    std::vector<BatchEntry> h_table;
    std::vector<int64_t> t_at_upload;
    std::vector<void *> cur_at_upload, nxt_at_upload;
    long long steps_since_upload, launches_since_upload;
    bool table_valid;
    int storage, force_on, coll;
    int fuse_max;             // steps per launch requested (1 or 2)
    int bx, rows;             // single-step shape
    int bx2, rows2;           // two-step shape
    bool auto_rows2;          // rows2 chosen at each upload (until autotuned)
    int total_tiles, total_tiles2;
    hipGraphExec_t graph;     // kGraphSteps batched steps, valid with the table
    bool graph_valid;
    std::string last_error;
};

namespace {

constexpr int kGraphSteps = 8;    // even: a multiple of the steps per launch
constexpr int kBatchRows2 = 24;   // segment rows of the two-step pass in a batch
const int kBatchRowsCand2[] = {2, 3, 4, 6, 8, 12, 16, 20, 24, 32, 40};

struct Layout {
    size_t err, diag_out, partials, rho_snap, bufA, bufB, total, plane, pitch;
    size_t r_off, r_pitch;  // per-cell mode: FP32 reference block after the populations
};

// Population storage, row-interleaved: row y of population i starts at
// element y * pitch + i * plane with plane = nx rounded up to 128 bytes and
// pitch = 9 plane.  Every row starts on a 128-byte boundary.  (On 2048 x 2048
// FP64 a 9-population stream in the kernel's walk order measured 6.3 TB/s in
// this layout against 6.0 TB/s with whole planes one after another.)  In the
// per-cell mode each buffer continues with the FP32 reference densities R,
// rows of nx rounded up to 128 bytes.
Layout layout_for(const lbm_params *p)
{
    Layout L;
    const size_t n = (size_t)p->nx * p->ny;
    const size_t es = elem_size(p->storage);
    L.plane = round_up((size_t)p->nx, 128 / es);
    L.pitch = kQ * L.plane;
    size_t off = 0;
    L.err = off;
    off += kAlign;
    L.diag_out = off;
    off += kAlign;
    L.partials = off;
    off += round_up((size_t)kMaxTiles * kDiag * sizeof(double), kAlign);
    L.rho_snap = off;
    off += round_up(n * sizeof(double), kAlign);
    L.r_off = round_up(L.pitch * p->ny * es, kAlign);
    L.r_pitch = round_up((size_t)p->nx, 32);
    const size_t buf =
        L.r_off + (p->storage == LBM_STORE_F16_LOCAL ? round_up(L.r_pitch * p->ny * 4, kAlign) : 0);
    L.bufA = off;
    off += buf;
    L.bufB = off;
    off += buf;
    L.total = off;
    return L;
}

bool params_valid(const lbm_params *p, std::string *why)
{
    auto fail = [&](const char *m) {
        if (why) *why = m;
        return false;
    };
    if (!p) return fail("params is NULL");
    if (p->nx < 3 || p->ny < 3) return fail("nx and ny must be >= 3");
    if ((double)p->nx * (double)p->ny >= 4294967296.0) return fail("nx*ny must be < 2^32");
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail("tau must be > 0.5");
    if (!(p->G != 0.0) || !std::isfinite(p->G)) return fail("G must be nonzero and finite");
    if (!std::isfinite(p->epsilon) || !std::isfinite(p->sigma)) return fail("eps/sigma not finite");
    if (!std::isfinite(p->eos_a) || !std::isfinite(p->eos_b) || !std::isfinite(p->eos_c) ||
        !std::isfinite(p->eos_k) || !std::isfinite(p->T))
        return fail("EOS constants not finite");
    if (p->force_on != 0 && p->force_on != 1) return fail("force_on must be 0 or 1");
    if (p->m2_trace_alt != 0 && p->m2_trace_alt != 1) return fail("m2_trace_alt must be 0 or 1");
    if (p->storage != LBM_STORE_F64 && p->storage != LBM_STORE_F32_SHIFTED &&
        p->storage != LBM_STORE_F16_SHIFTED && p->storage != LBM_STORE_F16_LOCAL)
        return fail("unknown storage mode");
    if (!std::isfinite(p->rho_ref)) return fail("rho_ref not finite");
    if (p->collision != LBM_COLL_BGK && p->collision != LBM_COLL_MRT)
        return fail("unknown collision operator");
    if (p->collision == LBM_COLL_MRT) {
        const double taus[5] = {p->tau_rho, p->tau_e, p->tau_zeta, p->tau_j, p->tau_q};
        for (double v : taus)
            if (!(v > 0.5) || !std::isfinite(v)) return fail("MRT relaxation times must be > 0.5");
    }
    return true;
}

Coeffs make_coeffs(const lbm_params *p, const Layout &L)
{
    const size_t pitch = L.pitch, plane = L.plane;
    Coeffs c;
    c.nx = p->nx;
    c.ny = p->ny;
    c.pitch = (int)pitch;
    c.plane = plane;
    c.omega = 1.0 / p->tau;
    c.guo = 1.0 - 1.0 / (2.0 * p->tau);
    c.eos_b = p->eos_b;
    c.kcT = p->eos_k * p->eos_c * p->T;
    c.ka = p->eos_k * p->eos_a;
    c.invG = 1.0 / p->G;
    c.cSC = -6.0 * p->G;
    c.cA = 9.0 * p->G * (1.5 * p->epsilon - p->sigma + 1.0);
    c.cB = 9.0 * p->G * (p->sigma - 1.0);
    c.rho_ref = (p->storage == LBM_STORE_F32_SHIFTED || p->storage == LBM_STORE_F16_SHIFTED)
                    ? p->rho_ref
                    : 0.0;
    c.r_off = L.r_off;
    c.r_pitch = (int)L.r_pitch;
    c.coll = p->collision;
    c.s_e = p->collision == LBM_COLL_MRT ? 1.0 / p->tau_e : 0.0;
    c.s_z = p->collision == LBM_COLL_MRT ? 1.0 / p->tau_zeta : 0.0;
    c.s_q = p->collision == LBM_COLL_MRT ? 1.0 / p->tau_q : 0.0;
    c.force_on = p->force_on;
    c.trace_alt = p->m2_trace_alt;
    c.storage = p->storage;
    return c;
}

// Strip width alignment in columns: 128 bytes of FP64, 64 bytes of FP32 or FP16.
int strip_align(int storage) { return is_f16(storage) ? 32 : 16; }

bool make_tiles(int nx, int ny, int bx, int seg_rows, int align, Tiles *tl,
                long long limit = kMaxTiles)
{
    int w = bx - 2;
    if (nx > w) w = w / align * align;
    else w = nx;
    if (w < 1) return false;
    tl->width = w;
    tl->nstrips = (nx + w - 1) / w;
    tl->nseg = (ny + seg_rows - 1) / seg_rows;
    const long long nt = (long long)tl->nstrips * tl->nseg;
    if (nt > limit) return false;
    tl->ntiles = (int)nt;
    return true;
}

// Tiles of the two-step pass: kHalo2 halo columns on each side of a strip.
bool make_tiles2(int nx, int ny, int bx, int seg_rows, int align, Tiles *tl)
{
    int w = bx - 2 * kHalo2;
    if (nx > w) w = w / align * align;
    else w = nx;
    if (w < 1) return false;
    tl->width = w;
    tl->nstrips = (nx + w - 1) / w;
    tl->nseg = (ny + seg_rows - 1) / seg_rows;
    const long long nt = (long long)tl->nstrips * tl->nseg;
    if (nt > kMaxTiles) return false;
    tl->ntiles = (int)nt;
    return true;
}

// Default launch shape: 256-thread workgroups unless another width wastes
// clearly fewer lanes on ragged strips (small lattices), then row segments
// short enough for about 64 waves per CU on 256 CUs (20 for FP16 storage, 28
// for FP16 with the per-cell reference), each segment at least 8 rows (FP64)
// or 5 rows (the others).  Many short segments keep more rows of loads in
// flight per CU (each segment starts with a burst of three row loads); their
// halo rows come back mostly from cache.
// Measured on 2048 x 2048 in sweeps over 128..512 threads and 3..25 rows:
// FP64 is fastest at (256 threads, 8 rows), FP32 at (256, 5..8), FP16 at
// (256, 16), FP16 with the per-cell reference at (256, 8..12).
void default_launch(int nx, int ny, int storage, int *bx_out, int *rows_out)
{
    int best = 256;
    double best_score = -1.0;
    const int align = strip_align(storage);
    for (int bx = 64; bx <= 512; bx += 64) {
        Tiles tl;
        if (!make_tiles(nx, ny, bx, 1 << 30, align, &tl)) continue;
        const double eff = (double)nx / ((double)tl.nstrips * bx);
        const double score = eff - (bx > 256 ? 0.1 : 0.0) + (bx == 256 ? 0.1 : 0.0);
        if (score > best_score + 1e-12) {
            best_score = score;
            best = bx;
        }
    }
    Tiles tb;
    make_tiles(nx, ny, best, 1 << 30, align, &tb);
    const double target_waves =
        256.0 * (storage == LBM_STORE_F16_SHIFTED ? 20.0 : (storage == LBM_STORE_F16_LOCAL ? 28.0 : 64.0));
    int nseg = (int)std::ceil(target_waves / ((double)tb.nstrips * (best / 64)));
    nseg = std::max(1, std::min(nseg, ny));
    int rows = (ny + nseg - 1) / nseg;
    rows = std::max(rows, std::min(storage == LBM_STORE_F64 ? 8 : 5, ny));
    while ((long long)tb.nstrips * ((ny + rows - 1) / rows) > kMaxTiles)
        ++rows;
    *bx_out = best;
    *rows_out = rows;
}

// Default shape of the two-step pass: 256 threads, and as many row segments
// as fill whole rounds of the workgroups the chip runs at once.  A workgroup
// walks its segment from start to end, so the launch takes as many rounds as
// it has tiles per concurrent slot, each about as long as a segment; a round
// that is only partly filled costs as much as a full one.  Slots per CU as
// measured best (FP64: two workgroups of 256 threads, VGPR-bound; FP32: two;
// FP16: four).  Segments have 2 to 40 rows: lattices too small to fill one
// round at 40 rows get one round of shorter segments (a lone workgroup is
// latency-bound, about 0.85 us per row), larger ones whole rounds of segments
// of up to 40 rows (longer ones gain nothing).  Measured, us per step, FP64:
// 2048^2 (256, 37) 67 against 72-89 for shapes that leave a partial round;
// 1024^2 11 rows 22.8 against 27.7 at 24; 64^2 2 rows 5.8 against 9.1 with
// single steps; 8192^2 32..64 rows within 1%.
constexpr int kFuseBx = 256;

int slots_per_cu2(int storage, int bx)
{
    const int per256 = is_f16(storage) ? 4 : 2;
    return std::max(1, per256 * 256 / bx);
}

// Segment length of the default two-step shape for block width bx on a chip
// with `cus` compute units.  False if no length fits kMaxTiles.
bool default_rows2(int nx, int ny, int storage, int bx, int cus, int *rows, Tiles *tl)
{
    const int min_rows = 2, max_rows = 40;
    Tiles t0;
    if (!make_tiles2(nx, ny, bx, ny, strip_align(storage), &t0)) return false;
    const long long slots = (long long)slots_per_cu2(storage, bx) * cus;
    const long long per_round = std::max(1ll, slots / t0.nstrips);  // segments per round
    long long nseg = per_round;
    if ((ny + nseg - 1) / nseg > max_rows)  // whole rounds of segments of <= max_rows
        nseg = per_round * ((ny + per_round * max_rows - 1) / (per_round * max_rows));
    if ((ny + nseg - 1) / nseg < min_rows) nseg = (ny + min_rows - 1) / min_rows;
    nseg = std::max(1ll, std::min<long long>(nseg, ny));
    for (int r = (int)((ny + nseg - 1) / nseg);; r = std::min(2 * r, ny)) {
        if (make_tiles2(nx, ny, bx, r, strip_align(storage), tl)) {
            *rows = r;
            return true;
        }
        if (r == ny) return false;
    }
}

// Compute units of the current device (256 on MI355X if the query fails).
int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        return 256;
    return cus;
}

lbm_status dev_fail(lbm_handle *h, hipError_t e, const char *what)
{
    if (h) {
        h->last_error = std::string(what) + ": " + hipGetErrorString(e);
    }
    return LBM_ERR_DEVICE;
}

template <int MODE, int FORCE, int ST, int COLL>
hipError_t launch_sweep_t(lbm_handle *h, const void *src, void *dst, Fields fo)
{
    const dim3 grid((unsigned)h->tiles.ntiles);
    const Coeffs &c = h->c;
    constexpr int PF = MODE == kStep ? kPrefetch : 1;
    switch (h->bx) {
#define LBM_CASE(BX)                                                                          \
    case BX:                                                                                  \
        hipLaunchKernelGGL((sweep_kernel<BX, MODE, PF, FORCE, ST, COLL>), grid, dim3(BX), 0,   \
                           h->stream, src, dst, c, h->tiles, (long long)h->t, h->err, fo,     \
                           h->rho_snap, h->partials);                                         \
        break;
        LBM_CASE(64)
        LBM_CASE(128)
        LBM_CASE(192)
        LBM_CASE(256)
        LBM_CASE(320)
        LBM_CASE(384)
        LBM_CASE(448)
        LBM_CASE(512)
#undef LBM_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int FORCE, int ST, int COLL>
hipError_t launch_sweep2_t(lbm_handle *h, const void *src, void *dst)
{
    const dim3 grid((unsigned)h->tiles2.ntiles);
    switch (h->bx2) {
#define LBM_CASE(BX)                                                                          \
    case BX:                                                                                  \
        hipLaunchKernelGGL((sweep2_kernel<BX, 1, FORCE, ST, COLL>), grid, dim3(BX), 0,         \
                           h->stream, src, dst, h->c, h->tiles2, (long long)h->t, h->err);    \
        break;
        LBM_CASE(128)
        LBM_CASE(256)
        LBM_CASE(512)
#undef LBM_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int FORCE, int ST>
hipError_t launch_sweep2_c(lbm_handle *h, const void *src, void *dst)
{
    return h->c.coll == LBM_COLL_MRT ? launch_sweep2_t<FORCE, ST, LBM_COLL_MRT>(h, src, dst)
                                     : launch_sweep2_t<FORCE, ST, LBM_COLL_BGK>(h, src, dst);
}

template <int FORCE>
hipError_t launch_sweep2_f(lbm_handle *h, const void *src, void *dst)
{
    switch (h->c.storage) {
    case LBM_STORE_F64: return launch_sweep2_c<FORCE, LBM_STORE_F64>(h, src, dst);
    case LBM_STORE_F32_SHIFTED: return launch_sweep2_c<FORCE, LBM_STORE_F32_SHIFTED>(h, src, dst);
    case LBM_STORE_F16_SHIFTED: return launch_sweep2_c<FORCE, LBM_STORE_F16_SHIFTED>(h, src, dst);
    case LBM_STORE_F16_LOCAL: return launch_sweep2_c<FORCE, LBM_STORE_F16_LOCAL>(h, src, dst);
    }
    return hipErrorInvalidValue;
}

// Two time steps, t -> t + 2, in one pass.
hipError_t launch_sweep2(lbm_handle *h, const void *src, void *dst)
{
    return h->c.force_on ? launch_sweep2_f<1>(h, src, dst) : launch_sweep2_f<0>(h, src, dst);
}

// The collision operator enters only the step sweep.
template <int MODE, int FORCE, int ST>
hipError_t launch_sweep_c(lbm_handle *h, const void *src, void *dst, Fields fo)
{
    if constexpr (MODE == kStep) {
        if (h->c.coll == LBM_COLL_MRT)
            return launch_sweep_t<MODE, FORCE, ST, LBM_COLL_MRT>(h, src, dst, fo);
    }
    return launch_sweep_t<MODE, FORCE, ST, LBM_COLL_BGK>(h, src, dst, fo);
}

template <int MODE, int FORCE>
hipError_t launch_sweep_f(lbm_handle *h, const void *src, void *dst, Fields fo)
{
    switch (h->c.storage) {
    case LBM_STORE_F64: return launch_sweep_c<MODE, FORCE, LBM_STORE_F64>(h, src, dst, fo);
    case LBM_STORE_F32_SHIFTED:
        return launch_sweep_c<MODE, FORCE, LBM_STORE_F32_SHIFTED>(h, src, dst, fo);
    case LBM_STORE_F16_SHIFTED:
        return launch_sweep_c<MODE, FORCE, LBM_STORE_F16_SHIFTED>(h, src, dst, fo);
    case LBM_STORE_F16_LOCAL:
        return launch_sweep_c<MODE, FORCE, LBM_STORE_F16_LOCAL>(h, src, dst, fo);
    }
    return hipErrorInvalidValue;
}

template <int MODE>
hipError_t launch_sweep(lbm_handle *h, const void *src, void *dst, Fields fo)
{
    return h->c.force_on ? launch_sweep_f<MODE, 1>(h, src, dst, fo)
                         : launch_sweep_f<MODE, 0>(h, src, dst, fo);
}

void launch_init(lbm_handle *h, unsigned blocks, const double *rho0, const double *ux0,
                 const double *uy0)
{
    switch (h->c.storage) {
    case LBM_STORE_F64:
        hipLaunchKernelGGL(init_kernel<LBM_STORE_F64>, dim3(blocks), dim3(256), 0, h->stream,
                           h->cur, h->c, rho0, ux0, uy0);
        break;
    case LBM_STORE_F32_SHIFTED:
        hipLaunchKernelGGL(init_kernel<LBM_STORE_F32_SHIFTED>, dim3(blocks), dim3(256), 0,
                           h->stream, h->cur, h->c, rho0, ux0, uy0);
        break;
    case LBM_STORE_F16_SHIFTED:
        hipLaunchKernelGGL(init_kernel<LBM_STORE_F16_SHIFTED>, dim3(blocks), dim3(256), 0,
                           h->stream, h->cur, h->c, rho0, ux0, uy0);
        break;
    default:
        hipLaunchKernelGGL(init_kernel<LBM_STORE_F16_LOCAL>, dim3(blocks), dim3(256), 0,
                           h->stream, h->cur, h->c, rho0, ux0, uy0);
        break;
    }
}

void launch_permute(lbm_handle *h, const void *in, void *out, int to_canonical)
{
    const size_t n = (size_t)h->p.nx * h->p.ny;
    const dim3 grid((unsigned)((n + 255) / 256));
    switch (h->c.storage) {
    case LBM_STORE_F64:
        hipLaunchKernelGGL(permute_kernel<LBM_STORE_F64>, grid, dim3(256), 0, h->stream, in,
                           out, h->c, to_canonical);
        break;
    case LBM_STORE_F32_SHIFTED:
        hipLaunchKernelGGL(permute_kernel<LBM_STORE_F32_SHIFTED>, grid, dim3(256), 0, h->stream,
                           in, out, h->c, to_canonical);
        break;
    case LBM_STORE_F16_SHIFTED:
        hipLaunchKernelGGL(permute_kernel<LBM_STORE_F16_SHIFTED>, grid, dim3(256), 0, h->stream,
                           in, out, h->c, to_canonical);
        break;
    default:
        hipLaunchKernelGGL(permute_kernel<LBM_STORE_F16_LOCAL>, grid, dim3(256), 0, h->stream,
                           in, out, h->c, to_canonical);
        break;
    }
}

lbm_status read_sticky(lbm_handle *h)
{
    unsigned long long key = ~0ull;
    hipError_t e = hipMemcpyAsync(&key, h->err, sizeof(key), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return dev_fail(h, e, "reading the error word");
    if (key != ~0ull) {
        const long long step = (long long)(key >> 32);
        const long long cell = (long long)(key & 0xffffffffull);
        char buf[160];
        std::snprintf(buf, sizeof buf,
                      "EOS domain left at step %lld, cell %lld (x=%lld, y=%lld)", step, cell,
                      cell % h->p.nx, cell / h->p.nx);
        h->last_error = buf;
        h->sticky = LBM_ERR_DOMAIN;
    }
    return h->sticky;
}


template <int FORCE, int ST, int COLL>
hipError_t launch_batch_t(lbm_batch *b)
{
    const dim3 grid((unsigned)b->total_tiles);
    const int nlat = (int)b->members.size();
    switch (b->bx) {
#define LBM_CASE(BX)                                                                          \
    case BX:                                                                                  \
        hipLaunchKernelGGL((batch_step_kernel<BX, kPrefetch, FORCE, ST, COLL>), grid, dim3(BX), \
                           0, b->stream, b->d_table, nlat, b->d_ctr);                         \
        break;
        LBM_CASE(64)
        LBM_CASE(128)
        LBM_CASE(192)
        LBM_CASE(256)
        LBM_CASE(320)
        LBM_CASE(384)
        LBM_CASE(448)
        LBM_CASE(512)
#undef LBM_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int FORCE, int ST>
hipError_t launch_batch_c(lbm_batch *b)
{
    return b->coll == LBM_COLL_MRT ? launch_batch_t<FORCE, ST, LBM_COLL_MRT>(b)
                                   : launch_batch_t<FORCE, ST, LBM_COLL_BGK>(b);
}

template <int FORCE>
hipError_t launch_batch_f(lbm_batch *b)
{
    switch (b->storage) {
    case LBM_STORE_F64: return launch_batch_c<FORCE, LBM_STORE_F64>(b);
    case LBM_STORE_F32_SHIFTED: return launch_batch_c<FORCE, LBM_STORE_F32_SHIFTED>(b);
    case LBM_STORE_F16_SHIFTED: return launch_batch_c<FORCE, LBM_STORE_F16_SHIFTED>(b);
    case LBM_STORE_F16_LOCAL: return launch_batch_c<FORCE, LBM_STORE_F16_LOCAL>(b);
    }
    return hipErrorInvalidValue;
}

// One batched step (the kernel only; the caller bumps the counters).
hipError_t launch_batch(lbm_batch *b)
{
    return b->force_on ? launch_batch_f<1>(b) : launch_batch_f<0>(b);
}

template <int FORCE, int ST, int COLL>
hipError_t launch_batch2_t(lbm_batch *b)
{
    const dim3 grid((unsigned)b->total_tiles2);
    const int nlat = (int)b->members.size();
    switch (b->bx2) {
#define LBM_CASE(BX)                                                                          \
    case BX:                                                                                  \
        hipLaunchKernelGGL((batch2_kernel<BX, 1, FORCE, ST, COLL>), grid, dim3(BX), 0,         \
                           b->stream, b->d_table, nlat, b->d_ctr);                            \
        break;
        LBM_CASE(128)
        LBM_CASE(256)
        LBM_CASE(512)
#undef LBM_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int FORCE, int ST>
hipError_t launch_batch2_c(lbm_batch *b)
{
    return b->coll == LBM_COLL_MRT ? launch_batch2_t<FORCE, ST, LBM_COLL_MRT>(b)
                                   : launch_batch2_t<FORCE, ST, LBM_COLL_BGK>(b);
}

template <int FORCE>
hipError_t launch_batch2_f(lbm_batch *b)
{
    switch (b->storage) {
    case LBM_STORE_F64: return launch_batch2_c<FORCE, LBM_STORE_F64>(b);
    case LBM_STORE_F32_SHIFTED: return launch_batch2_c<FORCE, LBM_STORE_F32_SHIFTED>(b);
    case LBM_STORE_F16_SHIFTED: return launch_batch2_c<FORCE, LBM_STORE_F16_SHIFTED>(b);
    case LBM_STORE_F16_LOCAL: return launch_batch2_c<FORCE, LBM_STORE_F16_LOCAL>(b);
    }
    return hipErrorInvalidValue;
}

// One batched two-step launch (the kernel only).
hipError_t launch_batch2(lbm_batch *b)
{
    return b->force_on ? launch_batch2_f<1>(b) : launch_batch2_f<0>(b);
}

// Steps per launch of a batch: two unless the caller has asked for single
// steps.
int batch_fuse(const lbm_batch *b) { return b->fuse_max; }

// One batched launch of `steps` (1 or 2) steps and its counter bump.
hipError_t batch_launch_steps(lbm_batch *b, int steps)
{
    hipError_t e = steps == 2 ? launch_batch2(b) : launch_batch(b);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(bump_counter, dim3(1), dim3(1), 0, b->stream, b->d_ctr,
                           (long long)steps);
        e = hipGetLastError();
    }
    return e;
}

// Average duration in microseconds of `reps` calls of fn on `stream`, after
// one untimed call.  Returns a negative value on a HIP error.
template <class Fn>
double time_launches(hipStream_t stream, int reps, Fn &&fn)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.0;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.0;
    }
    double us = -1.0;
    if (fn() == hipSuccess && hipEventRecord(e0, stream) == hipSuccess) {
        bool ok = true;
        for (int r = 0; r < reps && ok; ++r)
            ok = fn() == hipSuccess;
        float ms = 0.0f;
        if (ok && hipEventRecord(e1, stream) == hipSuccess &&
            hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
            us = 1e3 * ms / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return us;
}

const int kTuneWidths[] = {64, 128, 192, 256, 320, 384, 512};
const int kTuneRows[] = {3, 5, 7, 9, 13, 17};
const int kTuneWidths2[] = {128, 256, 512};
const int kTuneRows2[] = {12, 16, 20, 24, 32, 40, 48};

// Rebuild and upload the batch table for the current members and shape.
// Synchronous (the host staging vector is reused by the next upload).
lbm_status batch_upload(lbm_batch *b)
{
    b->h_table.clear();
    b->t_at_upload.clear();
    b->cur_at_upload.clear();
    b->nxt_at_upload.clear();
    int tile0 = 0, tile0_2 = 0;
    const int align = strip_align(b->storage);
    const bool two = batch_fuse(b) == 2;
    if (two && b->auto_rows2 && !b->members.empty()) {
        // the segment length that minimises rounds x (rows + 6) over the whole
        // batch, as for one lattice (the longer one on ties)
        const long long slots =
            (long long)slots_per_cu2(b->storage, b->bx2) * b->members[0]->cus;
        long long best = -1;
        for (int r : kBatchRowsCand2) {
            long long tiles = 0;
            bool ok = true;
            for (const lbm_handle *h : b->members) {
                Tiles t;
                if (!make_tiles2(h->p.nx, h->p.ny, b->bx2, std::min(r, h->p.ny), align, &t)) {
                    ok = false;
                    break;
                }
                tiles += t.ntiles;
            }
            if (!ok) continue;
            const long long cost = (tiles + slots - 1) / slots * (r + 6);
            if (best < 0 || cost <= best) {
                best = cost;
                b->rows2 = r;
            }
        }
    }
    for (lbm_handle *h : b->members) {
        BatchEntry e;
        e.c = h->c;
        if (!make_tiles(h->p.nx, h->p.ny, b->bx, std::min(b->rows, h->p.ny), align, &e.tl,
                        1ll << 30) ||
            (two && !make_tiles2(h->p.nx, h->p.ny, b->bx2, std::min(b->rows2, h->p.ny), align,
                                 &e.tl2))) {
            b->last_error = "launch shape does not fit a lattice of the batch";
            return LBM_ERR_INVALID_ARG;
        }
        if (!two) e.tl2 = Tiles{0, 0, 0, 0};
        e.buf[0] = h->cur;
        e.buf[1] = h->nxt;
        e.err = h->err;
        e.t0 = h->t;
        e.tile0 = tile0;
        e.tile0_2 = tile0_2;
        tile0 += e.tl.ntiles;
        tile0_2 += e.tl2.ntiles;
        b->h_table.push_back(e);
        b->t_at_upload.push_back(h->t);
        b->cur_at_upload.push_back(h->cur);
        b->nxt_at_upload.push_back(h->nxt);
    }
    b->total_tiles = tile0;
    b->total_tiles2 = tile0_2;
    hipError_t e = hipSuccess;
    if (!b->h_table.empty())
        e = hipMemcpyAsync(b->d_table, b->h_table.data(), b->h_table.size() * sizeof(BatchEntry),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(clear_counters, dim3(1), dim3(1), 0, b->stream, b->d_ctr);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        b->last_error = std::string("uploading the batch table: ") + hipGetErrorString(e);
        return LBM_ERR_DEVICE;
    }
    if (b->graph_valid) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph_valid = false;
    }
    b->steps_since_upload = 0;
    b->launches_since_upload = 0;
    b->table_valid = true;
    return LBM_OK;
}

// True when the table no longer describes the members: membership changed,
// or some member was stepped or restarted outside the batch since the table
// was written.
bool batch_stale(const lbm_batch *b)
{
    if (!b->table_valid || b->t_at_upload.size() != b->members.size()) return true;
    const bool odd = (b->launches_since_upload & 1) != 0;
    for (size_t k = 0; k < b->members.size(); ++k) {
        const lbm_handle *h = b->members[k];
        if (h->t != b->t_at_upload[k] + b->steps_since_upload) return true;
        if (h->cur != (odd ? b->nxt_at_upload[k] : b->cur_at_upload[k])) return true;
    }
    return false;
}

// Capture kGraphSteps batched steps (launches of batch_fuse(b) steps, each
// with its counter bump) in a graph.  An even number of launches, so a replay
// leaves every lattice's state in the buffer it started from.
hipError_t batch_capture(lbm_batch *b)
{
    hipGraph_t g;
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    const int per = batch_fuse(b);
    for (int k = 0; k < kGraphSteps / per && le == hipSuccess; ++k)
        le = batch_launch_steps(b, per);
    e = hipStreamEndCapture(b->stream, &g);
    if (le != hipSuccess) {
        if (e == hipSuccess) (void)hipGraphDestroy(g);
        return le;
    }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e == hipSuccess) b->graph_valid = true;
    return e;
}
}  // namespace

extern "C" {

size_t lbm_workspace_bytes(const lbm_params *params)
{
    if (!params_valid(params, nullptr)) return 0;
    return layout_for(params).total;
}

lbm_status lbm_init(const lbm_params *params, void *d_workspace, size_t workspace_bytes,
                    const double *d_rho0, const double *d_ux0, const double *d_uy0,
                    void *hip_stream, lbm_handle **out)
{
    if (!out) return LBM_ERR_INVALID_ARG;
    *out = nullptr;
    if (!params_valid(params, nullptr)) return LBM_ERR_INVALID_ARG;
    const Layout L = layout_for(params);
    if (!d_workspace || workspace_bytes < L.total || !d_rho0) return LBM_ERR_INVALID_ARG;
    if (((uintptr_t)d_workspace) % kAlign != 0) return LBM_ERR_INVALID_ARG;

    lbm_handle *h = new (std::nothrow) lbm_handle();
    if (!h) return LBM_ERR_OOM;
    h->p = *params;
    h->c = make_coeffs(params, L);
    h->stream = (hipStream_t)hip_stream;
    char *ws = (char *)d_workspace;
    h->err = (unsigned long long *)(ws + L.err);
    h->diag_out = (double *)(ws + L.diag_out);
    h->partials = (double *)(ws + L.partials);
    h->rho_snap = (double *)(ws + L.rho_snap);
    h->cur = (void *)(ws + L.bufA);
    h->nxt = (void *)(ws + L.bufB);
    h->t = 0;
    h->sticky = LBM_OK;
    default_launch(params->nx, params->ny, params->storage, &h->bx, &h->seg_rows);
    if (!make_tiles(params->nx, params->ny, h->bx, h->seg_rows, strip_align(params->storage),
                    &h->tiles)) {
        delete h;
        return LBM_ERR_INVALID_ARG;
    }
    // two steps per pass wherever a default shape fits
    h->cus = device_cus();
    h->bx2 = kFuseBx;
    h->fuse = default_rows2(params->nx, params->ny, params->storage, h->bx2, h->cus,
                            &h->seg_rows2, &h->tiles2)
                  ? 2
                  : 1;

    const size_t n = (size_t)params->nx * params->ny;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(fill_u64, dim3(1), dim3(1), 0, h->stream, h->err, ~0ull);
    launch_init(h, blocks, d_rho0, d_ux0, d_uy0);
    hipLaunchKernelGGL(copy_plane, dim3(blocks), dim3(256), 0, h->stream, d_rho0, h->rho_snap, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        delete h;
        return LBM_ERR_DEVICE;
    }
    *out = h;
    return LBM_OK;
}

lbm_status lbm_step(lbm_handle *h, int64_t nsteps)
{
    if (!h) return LBM_ERR_INVALID_ARG;
    if (nsteps < 0) {
        h->last_error = "nsteps must be >= 0";
        return LBM_ERR_INVALID_ARG;
    }
    int64_t k = 0;
    if (h->fuse == 2) {
        for (; k + 2 <= nsteps; k += 2) {
            hipError_t e = launch_sweep2(h, h->cur, h->nxt);
            if (e != hipSuccess) return dev_fail(h, e, "launching the two-step kernel");
            std::swap(h->cur, h->nxt);
            h->t += 2;
        }
    }
    for (; k < nsteps; ++k) {
        hipError_t e = launch_sweep<kStep>(h, h->cur, h->nxt, Fields{});
        if (e != hipSuccess) return dev_fail(h, e, "launching the step kernel");
        std::swap(h->cur, h->nxt);
        ++h->t;
    }
    return LBM_OK;
}

lbm_status lbm_sync(lbm_handle *h)
{
    if (!h) return LBM_ERR_INVALID_ARG;
    return read_sticky(h);
}

lbm_status lbm_moments(lbm_handle *h, double *d_rho, double *d_ux, double *d_uy, double *d_Fx,
                       double *d_Fy, double *d_psi)
{
    if (!h) return LBM_ERR_INVALID_ARG;
    Fields fo{d_rho, d_ux, d_uy, d_Fx, d_Fy, d_psi};
    hipError_t e = launch_sweep<kMoments>(h, h->cur, nullptr, fo);
    if (e != hipSuccess) return dev_fail(h, e, "launching the moments kernel");
    return read_sticky(h);
}

lbm_status lbm_diagnostics(lbm_handle *h, double out[6])
{
    if (!h || !out) return LBM_ERR_INVALID_ARG;
    hipError_t e = launch_sweep<kDiagnostics>(h, h->cur, nullptr, Fields{});
    if (e != hipSuccess) return dev_fail(h, e, "launching the diagnostics kernel");
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(256), 0, h->stream, h->partials,
                       h->tiles.ntiles, h->diag_out);
    e = hipGetLastError();
    if (e != hipSuccess) return dev_fail(h, e, "launching the reduction kernel");
    e = hipMemcpyAsync(out, h->diag_out, kDiag * sizeof(double), hipMemcpyDeviceToHost,
                       h->stream);
    if (e != hipSuccess) return dev_fail(h, e, "copying diagnostics");
    return read_sticky(h);
}

lbm_status lbm_get_populations(lbm_handle *h, double *d_f)
{
    if (!h || !d_f) return LBM_ERR_INVALID_ARG;
    launch_permute(h, h->cur, d_f, 1);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return dev_fail(h, e, "copying populations out");
    return LBM_OK;
}

lbm_status lbm_set_populations(lbm_handle *h, const double *d_f, int64_t t)
{
    if (!h || !d_f || t < 0) return LBM_ERR_INVALID_ARG;
    launch_permute(h, d_f, h->cur, 0);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return dev_fail(h, e, "copying populations in");
    h->t = t;
    return LBM_OK;
}

int64_t lbm_time(const lbm_handle *h) { return h ? h->t : -1; }

lbm_status lbm_set_launch(lbm_handle *h, int32_t block_x, int32_t seg_rows)
{
    if (!h) return LBM_ERR_INVALID_ARG;
    const int align = strip_align(h->p.storage);
    int dbx, drows;
    default_launch(h->p.nx, h->p.ny, h->p.storage, &dbx, &drows);
    const int bx = block_x != 0 ? block_x : dbx;
    const int rows = seg_rows != 0 ? seg_rows : drows;
    if (bx < 64 || bx > 512 || bx % 64 != 0 || rows < 1) {
        h->last_error = "block_x must be a multiple of 64 in [64, 512] and seg_rows >= 1";
        return LBM_ERR_INVALID_ARG;
    }
    Tiles tl;
    if (!make_tiles(h->p.nx, h->p.ny, bx, rows, align, &tl)) {
        h->last_error = "launch shape needs too many workgroups";
        return LBM_ERR_INVALID_ARG;
    }
    h->bx = bx;
    h->seg_rows = rows;
    h->tiles = tl;
    return LBM_OK;
}

lbm_status lbm_set_fusion(lbm_handle *h, int32_t steps, int32_t block_x, int32_t seg_rows)
{
    if (!h) return LBM_ERR_INVALID_ARG;
    if (steps == 1) {
        h->fuse = 1;
        return LBM_OK;
    }
    if (steps != 2) {
        h->last_error = "steps per pass must be 1 or 2";
        return LBM_ERR_INVALID_ARG;
    }
    const int bx = block_x != 0 ? block_x : kFuseBx;
    if ((bx != 128 && bx != 256 && bx != 512) || seg_rows < 0) {
        h->last_error = "block_x must be 128, 256 or 512 and seg_rows >= 1";
        return LBM_ERR_INVALID_ARG;
    }
    int rows = seg_rows;
    Tiles tl;
    if (rows == 0 ? !default_rows2(h->p.nx, h->p.ny, h->p.storage, bx, h->cus, &rows, &tl)
                  : !make_tiles2(h->p.nx, h->p.ny, bx, rows, strip_align(h->p.storage), &tl)) {
        h->last_error = "launch shape needs too many workgroups";
        return LBM_ERR_INVALID_ARG;
    }
    h->fuse = 2;
    h->bx2 = bx;
    h->seg_rows2 = rows;
    h->tiles2 = tl;
    return LBM_OK;
}

lbm_status lbm_get_launch(const lbm_handle *h, int32_t out[3])
{
    if (!h || !out) return LBM_ERR_INVALID_ARG;
    const bool two = h->fuse == 2;
    out[0] = two ? h->bx2 : h->bx;
    out[1] = two ? h->seg_rows2 : h->seg_rows;
    out[2] = two ? h->tiles2.ntiles : h->tiles.ntiles;
    return LBM_OK;
}

int32_t lbm_get_fusion(const lbm_handle *h) { return h ? h->fuse : -1; }

lbm_status lbm_autotune(lbm_handle *h, double out[3])
{
    if (!h) return LBM_ERR_INVALID_ARG;
    const int align = strip_align(h->p.storage);
    // single steps, always timed; launches cur -> nxt without swapping, so the
    // state is not advanced
    double best1 = 1e300;
    int bx1 = h->bx, rows1 = h->seg_rows;
    {
        const int bx0 = h->bx, rows0 = h->seg_rows;
        const Tiles tl0 = h->tiles;
        for (int bx : kTuneWidths)
            for (int rows : kTuneRows) {
                Tiles tl;
                if (!make_tiles(h->p.nx, h->p.ny, bx, std::min(rows, h->p.ny), align, &tl))
                    continue;
                h->bx = bx;
                h->seg_rows = std::min(rows, h->p.ny);
                h->tiles = tl;
                const double us = time_launches(h->stream, 3, [&] {
                    return launch_sweep<kStep>(h, h->cur, h->nxt, Fields{});
                });
                if (us < 0) {
                    h->bx = bx0;
                    h->seg_rows = rows0;
                    h->tiles = tl0;
                    return dev_fail(h, hipGetLastError(), "timing a launch shape");
                }
                if (us < best1) {
                    best1 = us;
                    bx1 = bx;
                    rows1 = h->seg_rows;
                }
            }
        make_tiles(h->p.nx, h->p.ny, bx1, rows1, align, &h->tiles);
        h->bx = bx1;
        h->seg_rows = rows1;
    }
    // the two-step pass, when in use (per time step: half a launch)
    double best2 = 1e300;
    int bx2 = h->bx2, rows2 = h->seg_rows2;
    if (h->fuse == 2) {
        const Tiles tl0 = h->tiles2;
        const int bx0 = h->bx2, rows0 = h->seg_rows2;
        for (int bx : kTuneWidths2)
            for (int k = -1; k < (int)(sizeof(kTuneRows2) / sizeof(int)); ++k) {
                // k = -1: the default segment length for this width
                Tiles tl;
                int r = 0;
                if (k < 0) {
                    if (!default_rows2(h->p.nx, h->p.ny, h->p.storage, bx, h->cus, &r, &tl))
                        continue;
                } else {
                    r = std::min(kTuneRows2[k], h->p.ny);
                    if (!make_tiles2(h->p.nx, h->p.ny, bx, r, align, &tl)) continue;
                }
                h->bx2 = bx;
                h->seg_rows2 = r;
                h->tiles2 = tl;
                const double us = time_launches(
                    h->stream, 3, [&] { return launch_sweep2(h, h->cur, h->nxt); });
                if (us < 0) {
                    h->bx2 = bx0;
                    h->seg_rows2 = rows0;
                    h->tiles2 = tl0;
                    return dev_fail(h, hipGetLastError(), "timing a launch shape");
                }
                if (0.5 * us < best2) {
                    best2 = 0.5 * us;
                    bx2 = bx;
                    rows2 = r;
                }
            }
        make_tiles2(h->p.nx, h->p.ny, bx2, rows2, align, &h->tiles2);
        h->bx2 = bx2;
        h->seg_rows2 = rows2;
        if (best1 < best2) h->fuse = 1;
    }
    if (out) {
        const bool two = h->fuse == 2;
        out[0] = two ? bx2 : bx1;
        out[1] = two ? rows2 : rows1;
        out[2] = two ? best2 : best1;  // per time step
    }
    return LBM_OK;
}

size_t lbm_batch_workspace_bytes(int32_t capacity)
{
    if (capacity < 1) return 0;
    return round_up((size_t)capacity * sizeof(BatchEntry), kAlign) + kAlign;
}

lbm_status lbm_batch_create(int32_t capacity, void *d_workspace, size_t workspace_bytes,
                            void *hip_stream, lbm_batch **out)
{
    if (!out) return LBM_ERR_INVALID_ARG;
    *out = nullptr;
    if (capacity < 1 || !d_workspace || workspace_bytes < lbm_batch_workspace_bytes(capacity) ||
        ((uintptr_t)d_workspace) % kAlign != 0)
        return LBM_ERR_INVALID_ARG;
    lbm_batch *b = new (std::nothrow) lbm_batch();
    if (!b) return LBM_ERR_OOM;
    b->capacity = capacity;
    b->stream = (hipStream_t)hip_stream;
    b->d_table = (BatchEntry *)d_workspace;
    b->d_ctr =
        (long long *)((char *)d_workspace + round_up((size_t)capacity * sizeof(BatchEntry), kAlign));
    b->steps_since_upload = 0;
    b->launches_since_upload = 0;
    b->table_valid = false;
    b->storage = -1;
    b->force_on = -1;
    b->coll = -1;
    b->fuse_max = 2;
    b->bx = 256;
    b->rows = 5;
    b->bx2 = 256;
    b->rows2 = kBatchRows2;
    b->auto_rows2 = true;
    b->total_tiles = 0;
    b->total_tiles2 = 0;
    b->graph_valid = false;
    *out = b;
    return LBM_OK;
}

lbm_status lbm_batch_add(lbm_batch *b, lbm_handle *h)
{
    if (!b || !h) return LBM_ERR_INVALID_ARG;
    if ((int)b->members.size() >= b->capacity) {
        b->last_error = "batch is full";
        return LBM_ERR_INVALID_ARG;
    }
    for (lbm_handle *m : b->members)
        if (m == h) return LBM_ERR_INVALID_ARG;
    if (!b->members.empty() &&
        (h->p.storage != b->storage || h->p.force_on != b->force_on ||
         h->p.collision != b->coll || h->stream != b->stream))
        return LBM_ERR_INVALID_ARG;
    if (b->members.empty()) {
        if (h->stream != b->stream) return LBM_ERR_INVALID_ARG;
        b->storage = h->p.storage;
        b->force_on = h->p.force_on;
        b->coll = h->p.collision;
    }
    b->members.push_back(h);
    b->table_valid = false;
    return LBM_OK;
}

lbm_status lbm_batch_remove(lbm_batch *b, lbm_handle *h)
{
    if (!b || !h) return LBM_ERR_INVALID_ARG;
    for (size_t k = 0; k < b->members.size(); ++k)
        if (b->members[k] == h) {
            b->members.erase(b->members.begin() + (long)k);
            b->table_valid = false;
            return LBM_OK;
        }
    return LBM_ERR_INVALID_ARG;
}

int32_t lbm_batch_size(const lbm_batch *b) { return b ? (int32_t)b->members.size() : -1; }

lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps)
{
    if (!b || nsteps < 0) return LBM_ERR_INVALID_ARG;
    if (b->members.empty() || nsteps == 0) return LBM_OK;
    if (batch_stale(b)) {
        const lbm_status st = batch_upload(b);
        if (st != LBM_OK) return st;
    }
    int64_t done = 0, launches = 0;
    const int per = batch_fuse(b);
    // the legacy null stream cannot be captured: there every launch is made
    // on its own
    const bool graphs = b->stream != nullptr;
    if (graphs && nsteps >= kGraphSteps && !b->graph_valid) {
        const hipError_t e = batch_capture(b);
        if (e != hipSuccess) {
            b->last_error = std::string("capturing the batch graph: ") + hipGetErrorString(e);
            return LBM_ERR_DEVICE;
        }
    }
    while (graphs && nsteps - done >= kGraphSteps) {
        const hipError_t e = hipGraphLaunch(b->graph, b->stream);
        if (e != hipSuccess) {
            b->last_error = std::string("launching the batch graph: ") + hipGetErrorString(e);
            return LBM_ERR_DEVICE;
        }
        done += kGraphSteps;
        launches += kGraphSteps / per;
    }
    while (done < nsteps) {
        const int k = nsteps - done >= per ? per : 1;
        const hipError_t e = batch_launch_steps(b, k);
        if (e != hipSuccess) {
            b->last_error = std::string("launching a batched step: ") + hipGetErrorString(e);
            return LBM_ERR_DEVICE;
        }
        done += k;
        ++launches;
    }
    b->steps_since_upload += nsteps;
    b->launches_since_upload += launches;
    for (lbm_handle *h : b->members) {
        h->t += nsteps;
        if (launches & 1) std::swap(h->cur, h->nxt);
    }
    return LBM_OK;
}

lbm_status lbm_batch_autotune(lbm_batch *b, double out[3])
{
    if (!b) return LBM_ERR_INVALID_ARG;
    if (b->members.empty()) return LBM_OK;
    const bool try_two = b->fuse_max == 2;
    // single steps, always timed (a batch of many small lattices can be
    // faster one step per launch); the counters stay 0 while timing, so every
    // timed launch reads the same buffers
    b->fuse_max = 1;
    double best1 = 1e300;
    int bx1 = b->bx, rows1 = b->rows;
    for (int bx : kTuneWidths)
        for (int rows : kTuneRows) {
            b->bx = bx;
            b->rows = rows;
            if (batch_upload(b) != LBM_OK) continue;
            const double us = time_launches(b->stream, 3, [&] { return launch_batch(b); });
            if (us >= 0 && us < best1) {
                best1 = us;
                bx1 = bx;
                rows1 = rows;
            }
        }
    b->bx = bx1;
    b->rows = rows1;
    double best2 = 1e300;
    int bx2 = b->bx2, rows2 = b->rows2;
    if (try_two) {
        b->fuse_max = 2;
        b->auto_rows2 = false;
        for (int bx : kTuneWidths2)
            for (int rows : kBatchRowsCand2) {
                b->bx2 = bx;
                b->rows2 = rows;
                if (batch_upload(b) != LBM_OK) continue;
                const double us =
                    0.5 * time_launches(b->stream, 3, [&] { return launch_batch2(b); });
                if (us >= 0 && us < best2) {
                    best2 = us;
                    bx2 = bx;
                    rows2 = rows;
                }
            }
        b->bx2 = bx2;
        b->rows2 = rows2;
    }
    const bool two = try_two && best2 <= best1;
    b->fuse_max = two ? 2 : 1;
    const lbm_status st = batch_upload(b);
    if (st != LBM_OK) return st;
    if (out) {
        out[0] = two ? bx2 : bx1;
        out[1] = two ? rows2 : rows1;
        out[2] = two ? best2 : best1;  // per time step
    }
    return LBM_OK;
}

lbm_status lbm_batch_set_fusion(lbm_batch *b, int32_t steps)
{
    if (!b || (steps != 1 && steps != 2)) return LBM_ERR_INVALID_ARG;
    if (steps != b->fuse_max) {
        b->fuse_max = steps;
        b->table_valid = false;  // the table holds the two-step tiles only when used
        if (b->graph_valid) {
            (void)hipGraphExecDestroy(b->graph);
            b->graph_valid = false;
        }
    }
    return LBM_OK;
}

int32_t lbm_batch_get_fusion(const lbm_batch *b) { return b ? batch_fuse(b) : -1; }

void lbm_batch_destroy(lbm_batch *b)
{
    if (!b) return;
    if (b->graph_valid) (void)hipGraphExecDestroy(b->graph);
    delete b;
}

const char *lbm_status_string(lbm_status s)
{
    switch (s) {
    case LBM_OK: return "ok";
    case LBM_ERR_INVALID_ARG: return "invalid argument";
    case LBM_ERR_DOMAIN: return "EOS domain error";
    case LBM_ERR_DEVICE: return "device error";
    case LBM_ERR_OOM: return "out of host memory";
    case LBM_ERR_STATE: return "invalid handle state";
    }
    return "unknown status";
}

const char *lbm_last_error(const lbm_handle *h) { return h ? h->last_error.c_str() : ""; }

void lbm_destroy(lbm_handle *h) { delete h; }

}  // extern "C"
