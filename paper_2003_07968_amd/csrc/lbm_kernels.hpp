#pragma once
// lbm_kernels.hpp -- device code of the D2Q9 force-approach pseudopotential
// lattice Boltzmann update for AMD CDNA4 (gfx950): storage formats, the
// per-cell arithmetic, the sweep kernels and their launchers.  The C ABI and
// the host runtime are in lbm.hip.
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

namespace lbmk {


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

inline size_t elem_size(int storage)
{
    return storage == LBM_STORE_F64 ? 8 : (storage == LBM_STORE_F32_SHIFTED ? 4 : 2);
}

inline bool is_f16(int storage)
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
// tr0, tr1, tr2: the trace M2_bb as tr0 psi_0 + tr1 (psi_1 + .. + psi_4) +
// tr2 (psi_5 + .. + psi_8), the direct trace of Eq. SOMED (-8, 1, 1)/27 or
// the alternative 2 cs^2 (M0 - psi_0) = (-10/27, 2/27, 1/54).
template <class R>
struct Phys {
    R omega, guo, eos_b, kcT, ka, invG, cSC, cA, cB, rho_ref, s_e, s_z, s_q;
    // Products of the coefficients above that the per-cell arithmetic uses,
    // formed once in FP64 and rounded to R (see rho_psi, force, collide).
    R g_kcT, g_ka, g_third;          // kcT/G, ka/G, 1/(3G)
    R m2_0, m2_1, m2_2, m2_58, m2_xy; // cA/9 times the M2 weights of s0, -s24, s13, s58, s5-s6
    R t0, t1, t2;                     // (cSC + cB tr0)/9, cB tr1/9, cB tr2/9
    R keep, om3, g3;                  // 1 - omega, omega/3, guo/3
    __device__ explicit Phys(const Coeffs &c)
        : omega((R)c.omega), guo((R)c.guo), eos_b((R)c.eos_b), kcT((R)c.kcT), ka((R)c.ka),
          invG((R)c.invG), cSC((R)c.cSC), cA((R)c.cA), cB((R)c.cB), rho_ref((R)c.rho_ref),
          s_e((R)c.s_e), s_z((R)c.s_z), s_q((R)c.s_q), g_kcT((R)(c.kcT * c.invG)),
          g_ka((R)(c.ka * c.invG)), g_third((R)(c.invG / 3.0)),
          m2_0((R)(c.cA * (-4.0 / 243.0))), m2_1((R)(c.cA * (-1.0 / 243.0))),
          m2_2((R)(c.cA * (2.0 / 243.0))), m2_58((R)(c.cA / 486.0)),
          m2_xy((R)(c.cA / 324.0)),
          t0((R)((c.cSC + c.cB * (c.trace_alt ? -10.0 / 27.0 : -8.0 / 27.0)) / 9.0)),
          t1((R)(c.cB * (c.trace_alt ? 2.0 / 27.0 : 1.0 / 27.0) / 9.0)),
          t2((R)(c.cB * (c.trace_alt ? 1.0 / 54.0 : 1.0 / 27.0) / 9.0)),
          keep((R)(1.0 - c.omega)), om3((R)(c.omega / 3.0)), g3((R)(c.guo / 3.0))
    {
    }
};

// Tile decomposition of one sweep.  Strip s covers interior columns
// [s * width, min(nx, (s + 1) * width)); whenever the lattice needs more than
// one strip, width is a multiple of 64 bytes of FP32 or FP16 or 128 bytes of
// FP64 (single-step sweeps, so that the stores of neighbouring workgroups
// never share a cache line) or of 16 columns (the two-step pass).
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
// column enters as a 32-bit byte offset, so each load and store is a single
// scalar-base + vector-offset global access.
struct Cols {
    uint32_t o, m, p;  // byte offsets of columns x, x - 1 (wrapped), x + 1 (wrapped)
};

// The column's byte offset, passed through an empty asm statement at each
// access.  Left alone, the compiler widens the loop-invariant offset to 64
// bits once, before the row loop, and then forms every address with a 64-bit
// vector add instead of the scalar-base + 32-bit vector-offset form of the
// global load and store (nine vector adds per row and step).
__device__ __forceinline__ uint32_t col_offset(uint32_t o)
{
    asm("" : "+v"(o));
    return o;
}

template <class E, class R>
__device__ __forceinline__ R ld(const E *__restrict__ row, uint32_t byte_off)
{
    return (R) * (const E *)((const char *)row + col_offset(byte_off));
}

// Row r of the per-cell mode's reference block.
__device__ __forceinline__ float *ref_row(const void *base, const Coeffs &c, int r)
{
    return (float *)((char *)base + c.r_off) + (size_t)r * c.r_pitch;
}

// The nine populations of one cell to row y of the storage (nontemporal).
template <class E>
__device__ __forceinline__ void store_pops(E *__restrict__ dst, const Coeffs &c, int y,
                                           uint32_t col, const E v[kQ])
{
    E *row = dst + (size_t)y * c.pitch;
#pragma unroll
    for (int i = 0; i < kQ; ++i)
        __builtin_nontemporal_store(v[i], (E *)((char *)(row + i * c.plane) + col_offset(col)));
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
    const float *row = ref_row(src, c, r);
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

// Reciprocal and quotient in the arithmetic type.  FP64: the hardware
// reciprocal estimate refined by two Newton steps (x <- x + x (1 - v x), each
// doubling the correct bits), and the quotient corrected once by its residual
// (q <- q + (a - b q) / b), within about one ulp of the rounded result and
// with a shorter dependent chain than the IEEE division sequence; the
// arguments are well scaled (rho and (1 - b rho)^3 inside the EOS domain).
// FP32: the hardware's single-instruction forms, whose error of about one ulp
// is far below the storage rounding of the reduced-precision modes.
__device__ __forceinline__ double recip(double v)
{
    double x = __builtin_amdgcn_rcp(v);
    x = fma(x, fma(-v, x, 1.0), x);
    return fma(x, fma(-v, x, 1.0), x);
}
__device__ __forceinline__ float recip(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double quot(double a, double b)
{
    const double x = recip(b);
    const double q = a * x;
    return fma(fma(-b, q, a), x, q);
}
__device__ __forceinline__ float quot(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
// Square root: FP64 from the hardware reciprocal-square-root estimate y,
// g = v y and h = y/2 refined together (r = 1/2 - g h; g += g r; h += h r),
// then g corrected twice by its residual (g += (v - g g) h), within about one
// ulp; v >= 0 here (the EOS domain check), and v = 0 gives 0.  FP32: the
// single-instruction form.
__device__ __forceinline__ double root(double v)
{
    const double y = __builtin_amdgcn_rsq(v);
    double g = v * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    g = fma(fma(-g, g, v), h, g);
    g = fma(fma(-g, g, v), h, g);
    return v > 0.0 ? g : v;
}
__device__ __forceinline__ float root(float v) { return __builtin_amdgcn_sqrtf(v); }

// Density (Eq. FD) and pseudopotential (Eqs. CSEOS, DED) from the stored
// deviations d_i = f_i - w_i rho_ref: rho = rho_ref + sum_i d_i.  Returns
// false when the density is outside the EOS domain (with FORCE = 0, when it
// is not positive and finite).
// FP64 arithmetic goes with FP64 storage, which keeps the populations
// themselves (reference density 0): the reference terms are left out there.
template <class R>
constexpr bool kNoRef = std::is_same_v<R, double>;

template <class R>
__device__ __forceinline__ R density(const R d[kQ], R ref)
{
    const R s = (((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7]))) + d[8];
    if constexpr (kNoRef<R>)
        return s;
    else
        return s + ref;
}

template <int FORCE, class R>
__device__ __forceinline__ bool rho_psi(const R d[kQ], R ref, const Phys<R> &P, R &rho, R &psi)
{
    rho = density<R>(d, ref);
    if (!FORCE) {
        psi = R(0);
        return rho > R(0) && rho < R(INFINITY);
    }
    // rad = (p(rho) - rho/3)/G with p = kcT rho num/(1 - br)^3 - ka rho^2,
    // as rho (kcT/G num/(1 - br)^3 - (ka/G rho + 1/(3G)))
    const R br = P.eos_b * rho;
    const R om = R(1) - br;
    const R num = fma(br, fma(br, om, R(1)), R(1));  // 1 + br + br^2 - br^3
    const R lin = fma(P.g_ka, rho, P.g_third);
    const R rad = rho * fma(P.g_kcT, quot(num, om * om * om), -lin);
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
// DFTCCC, DFTCST).  The moments with the D2Q9 weights:
//   M1_x = (s1 - s3)/9 + (s5 - s6 - s7 + s8)/36, M1_y likewise,
//   M2_xx = -4/27 s0 + 2/27 (s1 + s3) - 1/27 (s2 + s4) + 1/54 (s5 + .. + s8),
//   M2_yy likewise with x and y exchanged, M2_xy = (s5 - s6 + s7 - s8)/36,
//   tr = tr0 s0 + tr1 (s1 + .. + s4) + tr2 (s5 + .. + s8) (the trace of M2,
//   either Eq. SOMED's or the alternative weights),
//   F_a = cSC s0 M1_a + cA M1_b M2_ab + cB tr M1_a.
// Evaluated as F_a = G0 N_a + N_b Q_ab with N = 9 M1 = (s1 - s3) + (a - b)/4,
// Q = cA M2/9 and G0 = (cSC s0 + cB tr)/9, the constant factors folded into
// the weights (Phys), each combination of psi values with multiply-adds.
template <class R>
__device__ __forceinline__ void force(const R s[kQ], const Phys<R> &P, R &Fx, R &Fy)
{
    const R d13 = s[1] - s[3], d24 = s[2] - s[4];
    const R s13 = s[1] + s[3], s24 = s[2] + s[4];
    const R a57 = s[5] - s[7], b68 = s[6] - s[8];
    const R p57 = s[5] + s[7], p68 = s[6] + s[8];
    const R s58 = p57 + p68;
    const R Nx = fma(R(0.25), a57 - b68, d13);
    const R Ny = fma(R(0.25), a57 + b68, d24);
    const R q0 = fma(P.m2_0, s[0], P.m2_58 * s58);
    const R Qxx = fma(P.m2_2, s13, fma(P.m2_1, s24, q0));
    const R Qyy = fma(P.m2_2, s24, fma(P.m2_1, s13, q0));
    const R Qxy = (p57 - p68) * P.m2_xy;
    const R G0 = fma(P.t0, s[0], fma(P.t1, s13 + s24, P.t2 * s58));
    Fx = fma(G0, Nx, fma(Nx, Qxx, Ny * Qxy));
    Fy = fma(G0, Ny, fma(Nx, Qxy, Ny * Qyy));
}

// Velocity (Eq. FMD).  The w_i rho_ref parts of the populations carry no
// momentum, so the deviations give sum_i f_i c_i directly.
// J = rho u = sum_i f_i c_i + F/2 is returned too.
template <class R>
__device__ __forceinline__ void velocity(const R d[kQ], R rho, R Fx, R Fy, R &ux, R &uy, R &Jx,
                                         R &Jy)
{
    const R jx = ((d[1] - d[3]) + (d[5] - d[6])) + (d[8] - d[7]);
    const R jy = ((d[2] - d[4]) + (d[5] + d[6])) - (d[7] + d[8]);
    const R inv = recip(rho);
    Jx = fma(R(0.5), Fx, jx);
    Jy = fma(R(0.5), Fy, jy);
    ux = Jx * inv;
    uy = Jy * inv;
}

// BGK collision with the Guo source (Eqs. BGKCO, SEDF, GFS, GFSBGK), on the
// deviations d_i = f_i - w_i rho_ref, in place:
//   f^eq_i - w_i rho_ref = w_i ((rho - rho_ref) + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u))
//   S_i                  = (1 - 1/(2 tau)) w_i (3 c.F + 9 (c.F)(c.u) - 3 u.F)
//   d_i                 <- d_i + (f^eq_i - w_i rho_ref - d_i)/tau + S_i
// Gathered by powers of c_i, omega (f^eq_i - w_i rho_ref) + S_i =
// w_i [A + c_i.B + (c_i.u)(h c_i.u + m c_i.F)] with
//   A = omega (rho (1 - 3/2 u.u) - rho_ref) - 3 g u.F,  B = 3 (omega J + g F),
//   h = 9/2 omega rho,  m = 9 g,  g = 1 - 1/(2 tau),  J = rho u,
// and d_i <- (1 - omega) d_i + w_i [..].  Opposite directions share all but
// the sign of c_i.B: T = w (A + (c.u)(h c.u + m c.F)) once per pair, then
// d_i <- (1 - omega) d_i + T +- w c.B.  The diagonal weight is the axis
// weight / 4, an exact scaling.  Multiply-adds are written as explicit fma();
// the file is compiled without implicit contraction, so every inlined copy
// rounds the same way.
template <class R>
__device__ __forceinline__ void collide(R d[kQ], R ref, R rho, R ux, R uy, R Jx, R Jy, R Fx,
                                        R Fy, const Phys<R> &P)
{
    const R om = P.omega, g = P.guo, keep = P.keep;
    const R usq = fma(ux, ux, uy * uy);
    const R uF = fma(ux, Fx, uy * Fy);
    const R A = fma(om, fma(rho, R(-1.5) * usq, kNoRef<R> ? rho : rho - ref), R(-3) * g * uF);
    d[0] = fma(keep, d[0], R(4.0 / 9.0) * A);
    // axis directions (w = 1/9): w h = omega rho/2, w m = g, w B = (omega J + g F)/3
    const R A1 = R(1.0 / 9.0) * A;
    const R h1 = R(0.5) * om * rho;
    const R Bx = fma(P.om3, Jx, P.g3 * Fx), By = fma(P.om3, Jy, P.g3 * Fy);
    const R mx = g * Fx, my = g * Fy;
    const R Tx = fma(ux, fma(h1, ux, mx), A1);
    const R Ty = fma(uy, fma(h1, uy, my), A1);
    d[1] = fma(keep, d[1], Tx + Bx);
    d[3] = fma(keep, d[3], Tx - Bx);
    d[2] = fma(keep, d[2], Ty + By);
    d[4] = fma(keep, d[4], Ty - By);
    // diagonal directions (w = 1/36): directions 5/7 along (1, 1), 6/8 along (-1, 1)
    const R A2 = R(0.25) * A1, h2 = R(0.25) * h1;
    const R u5 = ux + uy, u6 = uy - ux;
    const R m5 = R(0.25) * (mx + my), m6 = R(0.25) * (my - mx);
    const R B5 = R(0.25) * (Bx + By), B6 = R(0.25) * (By - Bx);
    const R T5 = fma(u5, fma(h2, u5, m5), A2);
    const R T6 = fma(u6, fma(h2, u6, m6), A2);
    d[5] = fma(keep, d[5], T5 + B5);
    d[7] = fma(keep, d[7], T5 - B5);
    d[6] = fma(keep, d[6], T6 + B6);
    d[8] = fma(keep, d[8], T6 - B6);
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
    // lanes hold the tile's columns as a ring (see sweep_tile); neighbour
    // lanes are taken modulo BX, the two ends of the ring being the halo
    // columns, whose own results are not stored
    const int tx = threadIdx.x;
    const int txm = tx == 0 ? BX - 1 : tx - 1, txp = tx == BX - 1 ? 0 : tx + 1;
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
    const bool first = tx == BX - 1;  // column position 0, the left halo
    // the left neighbour of every lane but the first comes from the lane on
    // its left; the right neighbour was loaded (the first lane takes it from
    // the lane on its right)
    auto tri_of = [&](const RefPair<R> &v, float *buf) {
        buf[tx] = (float)v.own;
        __syncthreads();
        return first ? Tri<R>{v.side, v.own, (R)buf[txp]} : Tri<R>{(R)buf[txm], v.own, v.side};
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
        R ux, uy, Jx, Jy;
        velocity<R>(f[cur], C.rho, Fx, Fy, ux, uy, Jx, Jy);
        const size_t row = (size_t)y * c.nx;
        if (MODE == kStep) {
            if constexpr (COLL == LBM_COLL_MRT)
                collide_mrt<R>(f[cur], C.rho, ux, uy, Fx, Fy, P);
            else
                collide<R>(f[cur], ref_cur, C.rho, ux, uy, Jx, Jy, Fx, Fy, P);
            if (interior) {
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
                    E X[kQ];
#pragma unroll
                    for (int i = 0; i < kQ; ++i) {
                        const R w = i == 0 ? R(4.0 / 9.0) : (i < 5 ? R(1.0 / 9.0) : R(1.0 / 36.0));
                        const R dev = fma(-w, sd, g[i]);
                        X[i] = (E)dev;
                        err += dev - (R)X[i];
                    }
                    store_pops<E>(dst, c, y, cols.o, X);
                    float *rrow = ref_row(dst, c, y);
                    __builtin_nontemporal_store((float)(ref_cur + (sd + err)),
                                                (float *)((char *)rrow + col_offset(2 * cols.o)));
                } else {
                    E X[kQ];
#pragma unroll
                    for (int i = 0; i < kQ; ++i)
                        X[i] = (E)f[cur][i];
                    store_pops<E>(dst, c, y, cols.o, X);
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

    // lane tx holds column xs - 1 + pos: the interior columns in lanes
    // 0 .. width - 1 (each wave's stores start on a cache line of the aligned
    // strip), the right halo after them and the left halo in the last lane
    const int pos = (int)((threadIdx.x + 1) % BX);
    const int width = xe - xs;                 // interior columns, <= BX - 2
    const bool active = pos <= width + 1;
    const bool interior = pos >= 1 && pos <= width;
    int x = xs - 1 + (active ? pos : 1);
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
        if (threadIdx.x == 0) {
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

// A pointer read from the batch table, known to address global memory.
// Pointers loaded from memory are generic to the compiler, which addresses
// them with flat instructions (64-bit address arithmetic on the vector ALU,
// waits on both counters).  Rebuilt from its integer value as a pointer in
// the global address space, and only then widened to a generic one, it is
// inferred to be global at every use and gets the same global loads and
// stores as a kernel argument's pointer.
template <class T>
__device__ __forceinline__ T *as_global(T *p)
{
    using G = __attribute__((address_space(1))) T *;
    const G g = (G)(uintptr_t)p;
    return (T *)g;
}

// The fields of a lattice's batch entry that a launch uses, copied out of the
// table once per workgroup.
struct BatchTile {
    Coeffs c;
    Tiles tl;
    const void *src;
    void *dst;
    unsigned long long *err;
    long long t;
    int tile;
};
template <int BatchEntry::*F, Tiles BatchEntry::*TL>
__device__ __forceinline__ BatchTile batch_tile(const BatchEntry *__restrict__ table, int nlat,
                                                int b, long long steps, int parity)
{
    const BatchEntry &e = batch_entry<F>(table, nlat, b);
    return BatchTile{e.c,
                     e.*TL,
                     as_global(e.buf[parity]),
                     as_global(const_cast<void *>(e.buf[parity ^ 1])),
                     as_global(e.err),
                     e.t0 + steps,
                     b - e.*F};
}

// Where a batched launch starts: the steps and the launches since the batch
// table was written (the first gives the time, the parity of the second the
// source buffer).  Eager launches pass them as arguments (d_ctr = nullptr);
// launches captured in a graph add their position in the graph to counters
// in device memory, d_ctr[0] steps and d_ctr[1] launches, which a one-thread
// kernel at the end of the graph moves on, so that every replay starts where
// the previous one ended.
struct BatchPos {
    long long steps;
    int parity;
};
__device__ __forceinline__ BatchPos batch_pos(const long long *__restrict__ d_ctr,
                                              long long steps_add, int launches_add)
{
    const long long s0 = d_ctr ? d_ctr[0] : 0, l0 = d_ctr ? d_ctr[1] : 0;
    return BatchPos{s0 + steps_add, (int)((l0 + launches_add) & 1)};
}

// One time step of every lattice of a batch: workgroup b takes batch tile
// xcd_tile(b) and runs tile b - tile0 of its lattice; time and source buffer
// from batch_pos.
template <int BX, int PF, int FORCE, int ST, int COLL>
__global__ __launch_bounds__(BX, (kMinWaves<ST, COLL>)) void batch_step_kernel(
    const BatchEntry *__restrict__ table, int nlat, const long long *__restrict__ d_ctr,
    long long steps_add, int launches_add)
{
    const BatchPos pos = batch_pos(d_ctr, steps_add, launches_add);
    const BatchTile k = batch_tile<&BatchEntry::tile0, &BatchEntry::tl>(
        table, nlat, xcd_tile(blockIdx.x, gridDim.x), pos.steps, pos.parity);
    sweep_tile<BX, kStep, PF, FORCE, ST, COLL>(k.src, k.dst, k.c, k.tl, k.tile, k.t, k.err,
                                               Fields{}, nullptr, nullptr);
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
//   collides B's row m - 6, whose pulled populations it kept in registers
//   since the previous iteration, and stores it.
// psi rows live in LDS rings of three rows (slot = iteration mod 3); the
// force reads its 3 x 3 window there.  Of A's post-collision values only the
// populations that B pulls from a neighbouring lane go through LDS, each kept
// until B has pulled it: those pulled from the walk's next row (lattice row
// r + 1 walking up) for one iteration, 1 and 3 (row r) two, those pulled from
// the walk's previous row (r - 1 walking up) three.  Populations 0 and the
// two vertical ones come from the own lane and stay in registers.  Register
// sets rotate with period 6 (the loop is unrolled six times).
//
// Walk direction: neighbouring segments walk in opposite directions, as in the
// single-step sweep, so that the six rows two segments share (three halo rows
// of each) are read by both near the same time, at the start or at the end of
// both walks, and the second read comes from L2.  The hand-over buffers are
// named by their place in the walk, not by population: walking up, the
// previous row gives B populations 2, 5, 6 and the next row 4, 7, 8; walking
// down, the two sets trade places.  The direction is a template argument (one
// walk instantiated per direction), so both walks use the same rings and
// registers, and the two rows of the force stencil are picked at compile time
// too.  In the per-cell FP16 mode the reference rows that rebuild a row's
// deviations are taken in the same walk order and handed to the reconstruction
// in lattice order.
template <class R, int BX, bool LOC>
struct Pass2Lds {
    R psi_a[3][BX], psi_b[3][BX];  // psi of A's and B's rows
    // A's post-collision populations that B pulls from a neighbouring lane,
    // one slot per row that is still to be pulled
    R pa[2][BX];                   // diagonal pair from the walk's next row
    R p13[2][2][BX];               // populations 1, 3 of the current row
    R pb[3][2][BX];                // diagonal pair from the walk's previous row
    // per-cell mode: the reference R of A's input rows (exchanged for the
    // neighbours' values) and the new R of A's output rows (B reads it for
    // rows r - 1, r, r + 1)
    float r_in[LOC ? 2 : 1][BX], r_out[LOC ? 3 : 1][BX];
};

// Halo columns of the two-step pass on each side of its output strip.
constexpr int kHalo2 = 3;

template <int BX, int PF, int FORCE, int ST, int COLL, int DIR>
__device__ __forceinline__ void walk2(const typename Store<ST>::E *__restrict__ src,
                                      typename Store<ST>::E *__restrict__ dst, const Coeffs &c,
                                      long long t, int y0, int n, int x, const Cols &cols,
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
    // Lanes hold the tile's columns as a ring (see sweep2_tile): lane l holds
    // column position (l + kHalo2) mod BX, so the output columns start at
    // lane 0 and every wave stores whole cache lines.  Neighbour lanes are
    // taken modulo BX; the two ends of the ring are the outermost halo
    // columns, whose results no output uses.
    static_assert((BX & (BX - 1)) == 0, "ring of lanes needs a power-of-two width");
    const int tx = threadIdx.x;
    const int txm = (tx + BX - 1) & (BX - 1), txp = (tx + 1) & (BX - 1);
    // walk position s is lattice row y0 + DIR s (DIR = +1 or -1);
    // the direction is a template argument, so every choice below that
    // depends on it is made at compile time
    static_assert(DIR == 1 || DIR == -1, "a walk goes up or down the lattice");
    constexpr bool fwd = DIR > 0;
    constexpr int ystep = DIR;
    auto lrow = [&](int s) {
        const int r = (y0 + ystep * s) % c.ny;
        return r < 0 ? r + c.ny : r;
    };
    // psi ring slots of the rows on either side of the walk's current row,
    // as lattice rows r - 1 (dn) and r + 1 (up), from the slots of the walk's
    // previous (back) and next (ahead) rows
    auto slot_dn = [&](int back, int ahead) { return fwd ? back : ahead; };
    auto slot_up = [&](int back, int ahead) { return fwd ? ahead : back; };
    auto check = [&](bool ok, long long step, int s) {
        if (!ok) bad = min(bad, domain_key(step, lrow(s), x, c.nx));
    };
    // psi window row of slot s of a ring
    auto psi_row = [&](const R(*ring)[BX], int s) {
        return Row<R>{ring[s][txm], ring[s][tx], ring[s][txp], R(0)};
    };

    R fa[K][kQ];
    R rho_a[2], rho_b[2];   // rho of the last two psi rows of each step
    // population 0 and the vertical ones of A's last post-collision rows:
    // hb pulled from the walk's previous row (2 walking up, 4 walking down),
    // ha from its next row
    R h0[2], hb[3], ha;
    // populations B pulls from the walk's previous row (kB) and next row
    // (kA): the vertical one, then the diagonal pair in the order of their
    // LDS slots (previous row: from lane txm, from txp; next row: from txp,
    // from txm)
    constexpr int kB0 = fwd ? 2 : 4, kB1 = fwd ? 5 : 8, kB2 = fwd ? 6 : 7;
    constexpr int kA0 = fwd ? 4 : 2, kA1 = fwd ? 7 : 6, kA2 = fwd ? 8 : 5;
    // per-cell mode: R triples of A's input rows (slot = (row + 1) mod 3), R
    // of A's rows before their collision, R of the next rows in flight
    Tri<R> ta[3];
    R ra[2];
    RefPair<R> rl[2];
    // B's pulled populations of the row turned into psi (per-cell mode:
    // rebuilt as deviations from its R, kept in rb), held for the collision
    // of that row at the next iteration
    R gb[2][kQ];
    R rb[2];
    const bool first = tx == BX - kHalo2;  // column position 0, the leftmost
    // R at x - 1, x, x + 1 from a lane's own and side values and an LDS row
    auto tri_from = [&](const RefPair<R> &v, const float *buf) {
        return first ? Tri<R>{v.side, v.own, (R)buf[txp]} : Tri<R>{(R)buf[txm], v.own, v.side};
    };
    auto tri_lds = [&](const float *buf) {
        return Tri<R>{(R)buf[txm], (R)buf[tx], (R)buf[txp]};
    };
    // deviations from R triples given in walk order (previous, current, next
    // row), reconstruct taking them in lattice order (r - 1, r, r + 1)
    auto recon = [&](R g[kQ], const Tri<R> &back, const Tri<R> &cur, const Tri<R> &ahead) {
        if constexpr (fwd)
            reconstruct<R>(g, back, cur, ahead);
        else
            reconstruct<R>(g, ahead, cur, back);
    };
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            fa[k][i] = R(0);
    }
    rho_a[0] = rho_a[1] = rho_b[0] = rho_b[1] = R(0);
    hb[0] = hb[1] = hb[2] = R(0);
    h0[0] = h0[1] = R(0);
    ha = R(0);
    ra[0] = ra[1] = R(0);
    rb[0] = rb[1] = R(0);
#pragma unroll
    for (int i = 0; i < kQ; ++i)
        gb[0][i] = gb[1][i] = R(0);
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
                recon(fa[a_lead], ta[J % 3], ta[(J + 1) % 3], ta[(J + 2) % 3]);
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
                // walk rows m - 5 (back), m - 4 (current), m - 3 (ahead)
                const Row<R> D = psi_row(L.psi_a, slot_dn((J + 1) % 3, J % 3));
                const Row<R> C = psi_row(L.psi_a, (J + 2) % 3);
                const Row<R> U = psi_row(L.psi_a, slot_up((J + 1) % 3, J % 3));
                R sv[kQ];
                stencil<+1, R>(D, C, U, sv);
                force<R>(sv, P, Fx, Fy);
            }
            R *g = fa[a_cur];
            const R ref_cur = LOC ? ra[(J + 1) % 2] : gref;
            const R rho = rho_a[(J + 1) % 2];
            R ux, uy, Jx, Jy;
            velocity<R>(g, rho, Fx, Fy, ux, uy, Jx, Jy);
            if constexpr (COLL == LBM_COLL_MRT)
                collide_mrt<R>(g, rho, ux, uy, Fx, Fy, P);
            else
                collide<R>(g, ref_cur, rho, ux, uy, Jx, Jy, Fx, Fy, P);
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
                L.r_out[J % 3][tx] = (float)(ref_cur + (sd + err));
            }
            auto rd = [&](int i) { return LOC ? g[i] : (R)(E)g[i]; };
            h0[J % 2] = rd(0);
            hb[J % 3] = rd(kB0);
            ha = rd(kA0);
            L.p13[J % 2][0][tx] = rd(1);
            L.p13[J % 2][1][tx] = rd(3);
            L.pb[J % 3][0][tx] = rd(kB1);
            L.pb[J % 3][1][tx] = rd(kB2);
            L.pa[0][tx] = rd(kA1);
            L.pa[1][tx] = rd(kA2);
        }
        __syncthreads();
        // B's pulled populations of row m - 5, the row turned into psi now;
        // A's row q was written at iteration q + 4
        auto pull_b = [&](R g[kQ]) {
            // walk rows: ahead (written at m), current (m - 1, slot (J + 1) %
            // 2), back (m - 2, slot (J + 1) % 3); populations 4, 7, 8 come
            // from lattice row r + 1, 2, 5, 6 from r - 1, and a population
            // moving right (5, 8) from lane txm
            constexpr int sc = (J + 1) % 2, sb = (J + 1) % 3;
            g[kA0] = ha;
            g[kA1] = L.pa[0][txp];
            g[kA2] = L.pa[1][txm];
            g[kB0] = hb[sb];
            g[kB1] = L.pb[sb][0][txm];
            g[kB2] = L.pb[sb][1][txp];
            g[0] = h0[sc];
            g[1] = L.p13[sc][0][txm];
            g[3] = L.p13[sc][1][txp];
        };
        // step B: rho and psi of row m - 5
        if constexpr (DO_BPSI) {
            R *g = gb[J % 2];
            pull_b(g);
            R ref_b = gref;
            if constexpr (LOC) {
                // the walk's next, current and previous rows were handed
                // over at m, m - 1, m - 2
                const Tri<R> C = tri_lds(L.r_out[(J + 2) % 3]);
                recon(g, tri_lds(L.r_out[(J + 1) % 3]), C, tri_lds(L.r_out[J % 3]));
                ref_b = C.o;
                rb[J % 2] = ref_b;
            }
            R psi;
            const bool ok = rho_psi<FORCE, R>(g, ref_b, P, rho_b[J % 2], psi);
            if (valid_b && m - 5 >= -1) check(ok, t + 1, m - 5);
            L.psi_b[J % 3][tx] = psi;
        }
        __syncthreads();
        // step B: collision of row m - 6 and its store, from the populations
        // its psi pass pulled at the previous iteration
        if constexpr (DO_BCOL) {
            R g[kQ];
#pragma unroll
            for (int i = 0; i < kQ; ++i)
                g[i] = gb[(J + 1) % 2][i];
            const R ref_cur = LOC ? rb[(J + 1) % 2] : gref;
            R Fx = R(0), Fy = R(0);
            if (FORCE) {
                // walk rows m - 7 (back), m - 6 (current), m - 5 (ahead)
                const Row<R> D = psi_row(L.psi_b, slot_dn((J + 1) % 3, J % 3));
                const Row<R> C = psi_row(L.psi_b, (J + 2) % 3);
                const Row<R> U = psi_row(L.psi_b, slot_up((J + 1) % 3, J % 3));
                R sv[kQ];
                stencil<+1, R>(D, C, U, sv);
                force<R>(sv, P, Fx, Fy);
            }
            const R rho = rho_b[(J + 1) % 2];
            R ux, uy, Jx, Jy;
            velocity<R>(g, rho, Fx, Fy, ux, uy, Jx, Jy);
            if constexpr (COLL == LBM_COLL_MRT)
                collide_mrt<R>(g, rho, ux, uy, Fx, Fy, P);
            else
                collide<R>(g, ref_cur, rho, ux, uy, Jx, Jy, Fx, Fy, P);
            const int sb = m - 6;
            if (interior && sb >= 0 && sb < n) {
                const int yb = lrow(sb);
                if constexpr (LOC) {
                    // as the single-step store of the per-cell mode
                    const R sd =
                        (((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7]))) +
                        g[8];
                    R err = R(0);
                    E X[kQ];
#pragma unroll
                    for (int i = 0; i < kQ; ++i) {
                        const R w = i == 0 ? R(4.0 / 9.0) : (i < 5 ? R(1.0 / 9.0) : R(1.0 / 36.0));
                        const R dev = fma(-w, sd, g[i]);
                        X[i] = (E)dev;
                        err += dev - (R)X[i];
                    }
                    store_pops<E>(dst, c, yb, cols.o, X);
                    float *rrow = ref_row(dst, c, yb);
                    __builtin_nontemporal_store((float)(ref_cur + (sd + err)),
                                                (float *)((char *)rrow + col_offset(2 * cols.o)));
                } else {
                    E X[kQ];
#pragma unroll
                    for (int i = 0; i < kQ; ++i)
                        X[i] = (E)g[i];
                    store_pops<E>(dst, c, yb, cols.o, X);
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


// Waves per SIMD the two-step pass is compiled for.  FP64 runs at two (186
// VGPRs with BGK and the force, 38 kB of LDS per workgroup).  An earlier form
// of the pass was made to fit three (168 VGPRs with the density summed again
// at the collision and a few loop-invariant reloads) and gained nothing on
// 2048^2: the same 37-row segments measured the same, and the shorter
// segments that fill three slots per CU were slower (25 rows in one round:
// 130.6 against 125.6 us per launch), the pass being bound by the HBM access
// pattern rather than by latency.  The FP32-arithmetic modes fit four.
template <int ST>
constexpr int kWaves2 = ST == LBM_STORE_F64 ? 2 : 4;

// One tile of the two-step pass: output strip `strip` of row band `seg`; odd
// segments walk down the lattice (see walk2).
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
    // lane tx holds column xs - kHalo2 + pos: the output columns xs .. xe - 1
    // in lanes 0 .. width - 1 (so that each wave's stores start on a cache
    // line of an aligned strip), the right halo after them and the left halo
    // in the last kHalo2 lanes
    const int pos = (threadIdx.x + kHalo2) & (BX - 1);
    const int width = xe - xs;  // output columns, <= BX - 2 kHalo2
    const bool active = pos < width + 2 * kHalo2;
    const bool valid_b = pos >= kHalo2 - 1 && pos <= width + kHalo2;
    const bool interior = pos >= kHalo2 && pos < width + kHalo2;
    int x = (xs - kHalo2 + (active ? pos : kHalo2)) % c.nx;
    x = x < 0 ? x + c.nx : x;
    const int xm = wrap_lo(x - 1, c.nx), xp = wrap_hi(x + 1, c.nx);
    constexpr uint32_t es = sizeof(E);
    const Cols cols{(uint32_t)x * es, (uint32_t)xm * es, (uint32_t)xp * es};
    unsigned long long bad = ~0ull;
    if (seg & 1)
        walk2<BX, PF, FORCE, ST, COLL, -1>((const E *)src_v, (E *)dst_v, c, t, ye - 1, ye - ys,
                                           x, cols, active, valid_b, interior, lds, bad);
    else
        walk2<BX, PF, FORCE, ST, COLL, 1>((const E *)src_v, (E *)dst_v, c, t, ys, ye - ys, x,
                                          cols, active, valid_b, interior, lds, bad);
    if (bad != ~0ull) atomicMin(err, bad);
}

// The two-step pass over one lattice.
template <int BX, int PF, int FORCE, int ST, int COLL>
__global__ __launch_bounds__(BX) __attribute__((amdgpu_waves_per_eu(kWaves2<ST>)))
void sweep2_kernel(const void *__restrict__ src, void *__restrict__ dst, Coeffs c, Tiles tl,
                   long long t, unsigned long long *__restrict__ err)
{
    sweep2_tile<BX, PF, FORCE, ST, COLL>(src, dst, c, tl, xcd_tile(blockIdx.x, tl.ntiles), t, err);
}

// The two-step pass over every lattice of a batch (tiles and counters as in
// batch_step_kernel; a launch advances two steps and swaps the buffers once).
template <int BX, int PF, int FORCE, int ST, int COLL>
__global__ __launch_bounds__(BX) __attribute__((amdgpu_waves_per_eu(kWaves2<ST>)))
void batch2_kernel(const BatchEntry *__restrict__ table, int nlat,
                   const long long *__restrict__ d_ctr, long long steps_add, int launches_add)
{
    const BatchPos pos = batch_pos(d_ctr, steps_add, launches_add);
    const BatchTile k = batch_tile<&BatchEntry::tile0_2, &BatchEntry::tl2>(
        table, nlat, xcd_tile(blockIdx.x, gridDim.x), pos.steps, pos.parity);
    sweep2_tile<BX, PF, FORCE, ST, COLL>(k.src, k.dst, k.c, k.tl, k.tile, k.t, k.err);
}

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

// ---- Launchers ----------------------------------------------------------
//
// The host runtime (lbm.hip) reaches the kernels only through these
// functions.  Each is explicitly instantiated for one storage mode in a
// translation unit of its own (lbm_inst.hip, compiled once per storage mode
// and kernel family), so that the kernels of the four modes compile in
// parallel; every other unit sees only the extern declarations below.

// Arguments of a single-lattice sweep (single step, moments, diagnostics)
// or two-step pass; bx is the workgroup width.
struct SweepArgs {
    const void *src;
    void *dst;
    Coeffs c;
    Tiles tl;
    int bx;
    long long t;
    unsigned long long *err;
    Fields fo;
    double *rho_snap;
    double *partials;
    hipStream_t stream;
};

// Arguments of a batched launch: where it starts (batch_pos: counters in
// device memory, or nullptr, plus the steps and launches to add).
struct BatchArgs {
    const BatchEntry *table;
    int nlat;
    const long long *ctr;
    long long steps_add;
    int launches_add;
    int bx;
    unsigned grid;
    int force_on, coll;
    hipStream_t stream;
};

#define LBM_WIDTHS1(X) X(64) X(128) X(192) X(256) X(320) X(384) X(448) X(512)
#define LBM_WIDTHS2(X) X(128) X(256) X(512)

template <int MODE, int FORCE, int ST, int COLL>
hipError_t sweep_launch_bx(const SweepArgs &a)
{
    constexpr int PF = MODE == kStep ? kPrefetch : 1;
    const dim3 grid((unsigned)a.tl.ntiles);
    switch (a.bx) {
#define LBM_CASE(BX)                                                                          \
    case BX:                                                                                  \
        hipLaunchKernelGGL((sweep_kernel<BX, MODE, PF, FORCE, ST, COLL>), grid, dim3(BX), 0,   \
                           a.stream, a.src, a.dst, a.c, a.tl, a.t, a.err, a.fo, a.rho_snap,   \
                           a.partials);                                                       \
        break;
        LBM_WIDTHS1(LBM_CASE)
#undef LBM_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// One sweep of mode kStep (collision a.c.coll), kMoments or kDiagnostics.
template <int ST>
hipError_t launch_sweep(int mode, const SweepArgs &a)
{
    const bool mrt = a.c.coll == LBM_COLL_MRT;
    if (mode == kStep) {
        if (a.c.force_on)
            return mrt ? sweep_launch_bx<kStep, 1, ST, LBM_COLL_MRT>(a)
                       : sweep_launch_bx<kStep, 1, ST, LBM_COLL_BGK>(a);
        return mrt ? sweep_launch_bx<kStep, 0, ST, LBM_COLL_MRT>(a)
                   : sweep_launch_bx<kStep, 0, ST, LBM_COLL_BGK>(a);
    }
    if (mode == kMoments)
        return a.c.force_on ? sweep_launch_bx<kMoments, 1, ST, LBM_COLL_BGK>(a)
                            : sweep_launch_bx<kMoments, 0, ST, LBM_COLL_BGK>(a);
    return a.c.force_on ? sweep_launch_bx<kDiagnostics, 1, ST, LBM_COLL_BGK>(a)
                        : sweep_launch_bx<kDiagnostics, 0, ST, LBM_COLL_BGK>(a);
}

template <int FORCE, int ST, int COLL>
hipError_t sweep2_launch_bx(const SweepArgs &a)
{
    const dim3 grid((unsigned)a.tl.ntiles);
    switch (a.bx) {
#define LBM_CASE(BX)                                                                          \
    case BX:                                                                                  \
        hipLaunchKernelGGL((sweep2_kernel<BX, 1, FORCE, ST, COLL>), grid, dim3(BX), 0,         \
                           a.stream, a.src, a.dst, a.c, a.tl, a.t, a.err);                    \
        break;
        LBM_WIDTHS2(LBM_CASE)
#undef LBM_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Two time steps, t -> t + 2, in one pass.
template <int ST>
hipError_t launch_sweep2(const SweepArgs &a)
{
    const bool mrt = a.c.coll == LBM_COLL_MRT;
    if (a.c.force_on)
        return mrt ? sweep2_launch_bx<1, ST, LBM_COLL_MRT>(a)
                   : sweep2_launch_bx<1, ST, LBM_COLL_BGK>(a);
    return mrt ? sweep2_launch_bx<0, ST, LBM_COLL_MRT>(a)
               : sweep2_launch_bx<0, ST, LBM_COLL_BGK>(a);
}

template <int FORCE, int ST, int COLL>
hipError_t batch_launch_bx(const BatchArgs &a)
{
    switch (a.bx) {
#define LBM_CASE(BX)                                                                          \
    case BX:                                                                                  \
        hipLaunchKernelGGL((batch_step_kernel<BX, kPrefetch, FORCE, ST, COLL>), dim3(a.grid),  \
                           dim3(BX), 0, a.stream, a.table, a.nlat, a.ctr, a.steps_add,        \
                           a.launches_add);                                                   \
        break;
        LBM_WIDTHS1(LBM_CASE)
#undef LBM_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// One batched single step.
template <int ST>
hipError_t launch_batch(const BatchArgs &a)
{
    const bool mrt = a.coll == LBM_COLL_MRT;
    if (a.force_on)
        return mrt ? batch_launch_bx<1, ST, LBM_COLL_MRT>(a) : batch_launch_bx<1, ST, LBM_COLL_BGK>(a);
    return mrt ? batch_launch_bx<0, ST, LBM_COLL_MRT>(a) : batch_launch_bx<0, ST, LBM_COLL_BGK>(a);
}

template <int FORCE, int ST, int COLL>
hipError_t batch2_launch_bx(const BatchArgs &a)
{
    switch (a.bx) {
#define LBM_CASE(BX)                                                                          \
    case BX:                                                                                  \
        hipLaunchKernelGGL((batch2_kernel<BX, 1, FORCE, ST, COLL>), dim3(a.grid), dim3(BX), 0, \
                           a.stream, a.table, a.nlat, a.ctr, a.steps_add, a.launches_add);    \
        break;
        LBM_WIDTHS2(LBM_CASE)
#undef LBM_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// One batched two-step launch.
template <int ST>
hipError_t launch_batch2(const BatchArgs &a)
{
    const bool mrt = a.coll == LBM_COLL_MRT;
    if (a.force_on)
        return mrt ? batch2_launch_bx<1, ST, LBM_COLL_MRT>(a)
                   : batch2_launch_bx<1, ST, LBM_COLL_BGK>(a);
    return mrt ? batch2_launch_bx<0, ST, LBM_COLL_MRT>(a)
               : batch2_launch_bx<0, ST, LBM_COLL_BGK>(a);
}

// f(0) = f^eq(rho0, u0) into the population buffer X.
template <int ST>
hipError_t launch_init(void *X, const Coeffs &c, const double *rho0, const double *ux0,
                       const double *uy0, hipStream_t stream)
{
    const size_t n = (size_t)c.nx * c.ny;
    hipLaunchKernelGGL(init_kernel<ST>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       X, c, rho0, ux0, uy0);
    return hipGetLastError();
}

// Canonical FP64 f[9][ny][nx] <-> pull storage.
template <int ST>
hipError_t launch_permute(const void *in, void *out, const Coeffs &c, int to_canonical,
                          hipStream_t stream)
{
    const size_t n = (size_t)c.nx * c.ny;
    hipLaunchKernelGGL(permute_kernel<ST>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       stream, in, out, c, to_canonical);
    return hipGetLastError();
}

#define LBM_DECLARE_FAMILY1(EXT, ST)                                                          \
    EXT template hipError_t launch_sweep<ST>(int, const SweepArgs &);                         \
    EXT template hipError_t launch_batch<ST>(const BatchArgs &);                              \
    EXT template hipError_t launch_init<ST>(void *, const Coeffs &, const double *,           \
                                            const double *, const double *, hipStream_t);     \
    EXT template hipError_t launch_permute<ST>(const void *, void *, const Coeffs &, int,     \
                                               hipStream_t);
#define LBM_DECLARE_FAMILY2(EXT, ST)                                                          \
    EXT template hipError_t launch_sweep2<ST>(const SweepArgs &);                             \
    EXT template hipError_t launch_batch2<ST>(const BatchArgs &);
#define LBM_EXTERN extern
LBM_DECLARE_FAMILY1(LBM_EXTERN, LBM_STORE_F64)
LBM_DECLARE_FAMILY1(LBM_EXTERN, LBM_STORE_F32_SHIFTED)
LBM_DECLARE_FAMILY1(LBM_EXTERN, LBM_STORE_F16_SHIFTED)
LBM_DECLARE_FAMILY1(LBM_EXTERN, LBM_STORE_F16_LOCAL)
LBM_DECLARE_FAMILY2(LBM_EXTERN, LBM_STORE_F64)
LBM_DECLARE_FAMILY2(LBM_EXTERN, LBM_STORE_F32_SHIFTED)
LBM_DECLARE_FAMILY2(LBM_EXTERN, LBM_STORE_F16_SHIFTED)
LBM_DECLARE_FAMILY2(LBM_EXTERN, LBM_STORE_F16_LOCAL)
#undef LBM_EXTERN


}  // namespace lbmk
