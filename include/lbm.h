/*
 * lbm.h -- C ABI of the MI355X (gfx950) D2Q9 force-approach pseudopotential
 * lattice Boltzmann library.
 *
 * The method is that of Czelusniak, Mapelli, Guzella, Cabezas-Gomez and
 * Wagner, "Force approach for the pseudopotential lattice Boltzmann method"
 * (arXiv:2003.07968).  One time step (lbm_step) is, for every cell x of a
 * periodic nx * ny lattice:
 *
 *   1. streaming in pull form, f_i(x, t) = f*_i(x - c_i, t - 1)       (Eq. TLBE)
 *   2. density rho = sum_i f_i                                        (Eq. FD)
 *   3. pressure from the Carnahan-Starling EOS                        (Eq. CSEOS)
 *      P = k [c rho T (1 + b rho + (b rho)^2 - (b rho)^3)/(1 - b rho)^3 - a rho^2]
 *      and pseudopotential psi = sqrt((P - cs^2 rho)/G)                (Eq. DED)
 *   4. moments of w_i psi(x + c_i)                          (Eqs. FOMED, SOMED)
 *   5. the interaction force                                          (Eq. IFT)
 *      F = F^SC - (3/4) eps cs^2 G F^(1) + (sigma - 1) cs^2 G F^(2)
 *      with F^SC of Eq. SCF and F^(1), F^(2) of Eqs. DFTCCC, DFTCST
 *   6. velocity rho u = sum_i f_i c_i + F/2                           (Eq. FMD)
 *   7. BGK collision with the Guo source                (Eqs. BGKCO, GFS, GFSBGK)
 *      f*_i = f_i - (f_i - f_i^eq)/tau + (1 - 1/(2 tau)) w_i [c_i.F/cs^2
 *             + (c_ia c_ib - cs^2 d_ab) F_a u_b / cs^4],  f^eq of Eq. SEDF
 *      or the MRT collision with the Guo source      (Eqs. MRTCO, GFS, GFSMRT)
 *      f* = f - M^-1 Lambda M (f - f^eq) + M^-1 (I - Lambda/2) M s,
 *      with the Gram-Schmidt moment matrix M of Eq. MatrixMRT (Appendix A),
 *      Lambda of Eq. RelaxationMatrix and s the bracket of Eq. GFS
 *
 * with the D2Q9 velocities and weights of Sec. II.A (Eq. VelocitySet),
 * cs^2 = 1/3, in FP64 (or, with reduced-precision storage, FP32; see
 * lbm_storage).
 *
 * Conventions.
 *   - Every function is extern "C", returns an lbm_status (0 = LBM_OK) or a
 *     plain value, and never throws.
 *   - Pointers named d_* are HIP device pointers; everything else is host.
 *   - Fields are row-major [ny][nx], x fastest: cell (x, y) is y*nx + x.
 *   - Populations exchanged through the ABI are [9][ny][nx] in the order of
 *     Eq. VelocitySet (0 rest; 1..4 = +x, +y, -x, -y; 5..8 = (+,+), (-,+),
 *     (-,-), (+,-)) and hold f(t), the post-streaming, pre-collision state.
 *     The library's internal storage layout is private.
 *   - Ownership: the caller allocates and frees the device workspace and all
 *     device arrays; the library owns only the host-side handle.
 *   - Streams: all device work is enqueued, in order, on the HIP stream given
 *     to lbm_init (NULL = the null stream).  Calls on one handle must not
 *     overlap from several host threads.
 *   - Errors: bad arguments are rejected synchronously with
 *     LBM_ERR_INVALID_ARG and change nothing.  A density leaving the EOS domain
 *     (rho <= 0, b rho >= 1, (P - cs^2 rho)/G < 0 or non-finite) is recorded
 *     on the device in a sticky error word (first step, then lowest cell index);
 *     lbm_sync, lbm_moments and lbm_diagnostics then return LBM_ERR_DOMAIN and
 *     lbm_last_error names the step and cell.  The library never clamps psi.
 *     After a domain error the populations are undefined.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_ERR_INVALID_ARG = -1, /* rejected argument; nothing was changed        */
    LBM_ERR_DOMAIN = -2,      /* sticky: EOS domain left at some step and cell */
    LBM_ERR_DEVICE = -3,      /* a HIP call failed                              */
    LBM_ERR_OOM = -4,         /* host allocation failed                         */
    LBM_ERR_STATE = -5        /* handle not usable for this call                */
} lbm_status;

typedef enum {
    LBM_COLL_BGK = 0,          /* single relaxation time, Eq. BGKCO, Guo factor Eq. GFSBGK  */
    LBM_COLL_MRT = 1           /* multiple relaxation times, Eq. MRTCO, Guo factor
                                  Eq. GFSMRT, moment matrix of Eq. MatrixMRT               */
} lbm_collision;

typedef enum {
    LBM_STORE_F64 = 0,         /* populations stored in FP64, FP64 arithmetic           */
    LBM_STORE_F32_SHIFTED = 1, /* stored as FP32 deviations f_i - w_i rho_ref, FP32
                                  arithmetic (72 bytes per cell update)                */
    LBM_STORE_F16_SHIFTED = 2, /* stored as FP16 (IEEE binary16) deviations, FP32
                                  arithmetic (36 bytes per cell update)                */
    LBM_STORE_F16_LOCAL = 3    /* stored as FP16 deviations from w_i R(z), where R(z) is
                                  a per-cell FP32 reference density of the sending cell
                                  z: R = sum_i f*_i, X_i = round16(f*_i - w_i R), then R
                                  corrected by the nine rounding errors and rounded to
                                  FP32, so that the cell's mass is kept to FP32
                                  rounding; FP32 arithmetic (44 bytes per cell update:
                                  9 x 2 + 4 read, as much written).  rho_ref is not
                                  used.                                                */
} lbm_storage;

/* Physical and numerical parameters, named as in the paper. */
typedef struct {
    int32_t nx, ny;   /* periodic lattice, each >= 3                               */
    double tau;       /* BGK relaxation time, > 0.5 (Eq. BGKCO)                    */
    double G;         /* nonzero; sign and scale of Eq. DED.  The force depends
                         only on its sign (psi scales as |G|^-1/2).               */
    double epsilon;   /* coexistence parameter of Eq. IFT (paper: 1.73)            */
    double sigma;     /* surface-tension parameter of Eq. IFT (paper: 1/8 .. 4)    */
    double eos_a, eos_b, eos_c, eos_k; /* Eq. CSEOS constants                      */
    double T;         /* absolute temperature of Eq. CSEOS                         */
    int32_t force_on; /* 0: F = 0, plain BGK; 1: the force of Eq. IFT              */
    int32_t m2_trace_alt; /* 0: M2_bb as the trace of Eq. SOMED; 1: the
                             alternative 2 cs^2 (M0 - psi) stated after Eq. DFTCST */
    int32_t storage;  /* lbm_storage.  In the shifted modes each population is kept
                         as d_i = f_i - w_i rho_ref rounded to the storage type
                         (round to nearest even) after every step; density,
                         force, velocity and collision are evaluated in FP32 from
                         them.  Diagnostics sums stay FP64.                      */
    double rho_ref;   /* reference density of the shifted modes (normally the mean
                         initial density); ignored for LBM_STORE_F64              */
    int32_t collision; /* lbm_collision                                            */
    double tau_rho, tau_e, tau_zeta, tau_j, tau_q;
                      /* MRT relaxation times of Eq. RelaxationMatrix, each > 0.5:
                         Lambda = diag(1/tau_rho, 1/tau_e, 1/tau_zeta, 1/tau_j,
                         1/tau_q, 1/tau_j, 1/tau_q, 1/tau, 1/tau) on the moments
                         (rho, e, zeta, j_x, q_x, j_y, q_y, p_xx, p_xy); the stress
                         rows relax with tau, which sets the viscosity
                         cs^2 (tau - 1/2).  The mass and momentum rows are
                         conserved by the collision with the Guo source, so
                         tau_rho and tau_j do not change the result.  Ignored
                         for LBM_COLL_BGK.                                       */
} lbm_params;

typedef struct lbm_handle lbm_handle;

/* Bytes of device workspace lbm_init needs for these parameters (0 if they are
 * invalid).  The workspace holds two population copies (2 * 9 * nx * ny
 * elements of the storage type, rows padded to 128 bytes; with
 * LBM_STORE_F16_LOCAL each copy also holds nx * ny FP32 reference densities),
 * a density snapshot for the steady-state criterion (FP64), 1.5 MB of
 * reduction scratch and the error word. */
size_t lbm_workspace_bytes(const lbm_params *params);

/* Validate params, carve the workspace (device memory of at least
 * lbm_workspace_bytes, 256-byte aligned, owned by the caller and kept alive
 * until lbm_destroy) and set t = 0 with f(0) = f^eq(rho0, u0) (Sec. IV.A,
 * below Eq. ISD).  d_rho0 is [ny][nx]; d_ux0 and d_uy0 may be NULL (zero
 * velocity).  hip_stream is a hipStream_t.  On success *out receives a new
 * handle.  The initial density must lie in the EOS domain; that is checked
 * by the first step or moments call, not here. */
lbm_status lbm_init(const lbm_params *params, void *d_workspace, size_t workspace_bytes,
                    const double *d_rho0, const double *d_ux0, const double *d_uy0,
                    void *hip_stream, lbm_handle **out);

/* Enqueue nsteps >= 0 time steps (asynchronous).  Returns LBM_ERR_DEVICE if a
 * launch fails; domain errors surface at lbm_sync. */
lbm_status lbm_step(lbm_handle *h, int64_t nsteps);

/* Wait for the handle's stream and return the sticky status. */
lbm_status lbm_sync(lbm_handle *h);

/* Macroscopic fields at the current time t: rho (Eq. FD), u (Eq. FMD), the
 * force F (Eq. IFT, zero when force_on = 0) and psi (Eq. DED, zero when
 * force_on = 0).  Each output is a device array [ny][nx] or NULL to skip it.
 * Synchronous: returns after the fields are written, with the sticky status. */
lbm_status lbm_moments(lbm_handle *h, double *d_rho, double *d_ux, double *d_uy, double *d_Fx,
                       double *d_Fy, double *d_psi);

/* Global diagnostics at time t into host out[6]:
 *   out[0] mass, sum rho
 *   out[1], out[2] momentum, sum rho u_x and sum rho u_y (= sum f c + F/2)
 *   out[3] sum |rho(t) - rho_snap|, out[4] sum |rho(t)|: the numerator and
 *          denominator of the steady-state criterion (Eq. SSC), where rho_snap
 *          is the density at the previous lbm_diagnostics call (or at t = 0)
 *   out[5] max |u|
 * The call then replaces rho_snap by rho(t).  Sums are reduced in a fixed
 * order (deterministic for a given lattice size).  Synchronous. */
lbm_status lbm_diagnostics(lbm_handle *h, double out[6]);

/* For callers that cannot allocate device memory or that must not depend on
 * the workspace's reduction scratch (code that runs where hipMalloc is not
 * allowed, tight serving loops): lbm_diagnostics with its per-workgroup
 * partial sums and reduced values in a statically allocated device array of
 * the library instead.  Same results, bitwise, as lbm_diagnostics on the
 * same state (same kernels, same reduction order), and the same update of
 * the steady-state snapshot, which stays in the handle's workspace.
 *   - Allocates nothing: no hipMalloc, hipFree or allocating library call.
 *     The array holds the partials of at most 16384 workgroups of the
 *     diagnostics sweep plus six values (about 786 kB per device, held until
 *     the process ends).  The default shapes stay far below that; a lattice
 *     whose sweep needs more workgroups (very short segments set with
 *     lbm_set_launch) is rejected with LBM_ERR_INVALID_ARG, nothing is
 *     launched, and lbm_last_error says why.
 *   - Every call on one GPU uses that GPU's single array: calls that overlap
 *     on one GPU (from several host threads, or on several streams before
 *     the earlier call has returned) race and must be serialised by the
 *     caller.  The call is synchronous, so calls from one thread never
 *     overlap.
 *   - The handle's device (current at lbm_init) is made current for the
 *     call and the caller's current device restored afterwards. */
lbm_status lbm_diagnostics_noalloc(lbm_handle *h, double out[6]);

/* Copy f(t) out to d_f ([9][ny][nx] FP64, device).  Synchronous.  With shifted
 * storage the values are w_i rho_ref + d_i, exactly. */
lbm_status lbm_get_populations(lbm_handle *h, double *d_f);

/* Replace the state by f(t) = d_f ([9][ny][nx] FP64, device) and set the
 * time counter to t >= 0 (checkpoint restart).  With shifted storage each
 * f_i - w_i rho_ref is rounded to the storage type, so a state read with
 * lbm_get_populations comes back bitwise.  With LBM_STORE_F16_LOCAL each
 * cell's nine values are encoded afresh against their own sum; the rounded
 * deviations of a stored state need not sum to zero, so a value may move by
 * about one binary16 rounding of its deviation (restart close, not bitwise).
 * Synchronous.  Clears nothing else: a sticky error stays. */
lbm_status lbm_set_populations(lbm_handle *h, const double *d_f, int64_t t);

/* Number of completed steps. */
int64_t lbm_time(const lbm_handle *h);

/* Override the launch shape of the single-step sweep kernels (the moments and
 * diagnostics sweeps, and lbm_step when it takes single steps): block_x
 * threads per workgroup (a multiple of 64 in [64, 512]; each workgroup owns
 * block_x - 2 columns) and seg_rows rows walked by each workgroup (>= 1).  0
 * keeps the library's choice.  Every shape gives bitwise-identical
 * populations. */
lbm_status lbm_set_launch(lbm_handle *h, int32_t block_x, int32_t seg_rows);

/* Time steps per pass of the step kernel, 1 or 2.  With 2, lbm_step advances
 * pairs of steps in one pass that reads and writes the populations once: each
 * workgroup computes the first step (time t) on its tile and a halo of three
 * columns and three rows on each side, keeps it on chip, and computes and
 * stores the second (time t + 1) on its tile; an odd remainder takes a single
 * step.  The results are bitwise those of single steps (the state between the
 * two is rounded to the storage type as a single step stores it), and so is
 * the first domain error reported by lbm_sync.  block_x (128, 256 or 512;
 * each workgroup owns block_x - 6 columns, rounded down to the strip
 * alignment) and seg_rows (>= 1) set the two-step launch shape; 0 keeps the
 * library's choice (256 threads; segments of 2..40 rows, as many as fill whole
 * rounds of the workgroups the device runs at once).  lbm_init selects 2.
 * Batches have their own setting (lbm_batch_set_fusion). */
lbm_status lbm_set_fusion(lbm_handle *h, int32_t steps, int32_t block_x, int32_t seg_rows);

/* Time steps per pass in use (1 or 2); -1 for a NULL handle. */
int32_t lbm_get_fusion(const lbm_handle *h);

/* The launch shape of the step kernel in use (the two-step pass's when
 * lbm_get_fusion is 2): out[0] = block_x, out[1] = seg_rows, out[2] =
 * workgroups per launch. */
lbm_status lbm_get_launch(const lbm_handle *h, int32_t out[3]);

/* Pick the step kernel's launch shape by measurement: time a few launches for
 * each candidate shape (single steps: workgroup widths 64..512, segments of
 * 3..17 rows; two-step pass, when lbm_get_fusion is 2: widths 128, 256, 512,
 * each with its default segment length and segments of 12..48 rows) and keep
 * the fastest per time step, switching to single steps if they win (results
 * are bitwise the same; lbm_get_fusion tells which).  The timed launches
 * write only the spare population buffer and are not counted as steps, so
 * the state and t are unchanged.  Synchronous; out (may be NULL) receives the
 * chosen block_x, seg_rows and the measured microseconds per time step. */
lbm_status lbm_autotune(lbm_handle *h, double out[3]);

/* ---- Batches: many lattices advanced together by one kernel launch ----
 *
 * A batch holds up to `capacity` handles created by lbm_init on the same HIP
 * stream, all with the same storage mode, force_on and collision, any sizes
 * and any other parameters.  lbm_batch_step launches one kernel per two time
 * steps (the two-step pass; one per step after lbm_batch_set_fusion(b, 1),
 * and for an odd last step) covering every tile
 * of every lattice (a workgroup finds its lattice in a device table), and
 * replays a captured HIP graph of eight steps for every full eight steps of a
 * call (not on the legacy null stream, which cannot be captured: there each
 * launch is made on its own).  Each lattice keeps its own workspace, state,
 * time counter and sticky error word, so lbm_moments, lbm_diagnostics,
 * lbm_sync and checkpointing work per handle as before, and results are
 * bitwise the same as stepping the handle alone.  A member may also be
 * stepped or restarted on its own between batch calls: the next
 * lbm_batch_step notices and rewrites the table (a synchronous upload), as it
 * does after lbm_batch_add or lbm_batch_remove. */
typedef struct lbm_batch lbm_batch;

/* Device bytes of the batch table for `capacity` lattices. */
size_t lbm_batch_workspace_bytes(int32_t capacity);

/* Create an empty batch; d_workspace (>= lbm_batch_workspace_bytes, 256-byte
 * aligned, caller-owned) holds the device table.  hip_stream must be the
 * stream of the handles that will be added. */
lbm_status lbm_batch_create(int32_t capacity, void *d_workspace, size_t workspace_bytes,
                            void *hip_stream, lbm_batch **out);

/* Add or remove a handle (the handle stays owned by the caller).  Adding fails
 * with LBM_ERR_INVALID_ARG if the batch is full, the handle is already in it,
 * or its storage mode, force_on, collision or stream differ from the batch's. */
lbm_status lbm_batch_add(lbm_batch *b, lbm_handle *h);
lbm_status lbm_batch_remove(lbm_batch *b, lbm_handle *h);
int32_t lbm_batch_size(const lbm_batch *b);

/* Advance every lattice of the batch by nsteps (asynchronous). */
lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps);

/* Choose the batch's workgroup width and segment length by timing candidate
 * shapes on the batch as it is (state unchanged, as lbm_autotune): single
 * steps, and the two-step pass unless lbm_batch_set_fusion(b, 1) was called
 * (each width's default length and segments of 2..40 rows).  Every shape is
 * timed over a few launches, the fastest three again over longer samples;
 * the faster form per time step is kept (lbm_batch_get_fusion tells which).
 * Shapes within about 1% of each other may swap places between calls.
 * Synchronous; out (may be NULL): block_x, seg_rows, microseconds per time
 * step. */
lbm_status lbm_batch_autotune(lbm_batch *b, double out[3]);

/* Time steps per batched launch: 2 (the default) or 1.  Results are bitwise
 * the same either way.  The next lbm_batch_step rewrites the table.
 * Until lbm_batch_autotune or lbm_batch_set_launch is called, the two-step
 * segment length is chosen at each table upload to fill whole rounds of the
 * workgroups the device runs at once (2..48 rows over all members). */
lbm_status lbm_batch_set_fusion(lbm_batch *b, int32_t steps);

/* Steps per batched launch in use (1 or 2; -1 for NULL). */
int32_t lbm_batch_get_fusion(const lbm_batch *b);

/* Fix the batch's launch: `steps` per launch (1 or 2) with workgroups of
 * block_x threads walking segments of seg_rows rows.  Two-step pass: block_x
 * 128, 256 or 512, seg_rows >= 1, or 0 for the length chosen at each table
 * upload (as before lbm_batch_autotune).  Single steps: block_x a multiple of
 * 64 in 64..512, seg_rows >= 1.  Other values: LBM_ERR_INVALID_ARG, nothing
 * changed.  For callers that have measured a shape (lbm_batch_autotune) and
 * want it again without the timing, and for profiling runs that must launch
 * one known shape.  Results are bitwise the same for every shape.  The next
 * lbm_batch_step rewrites the table; a shape that needs more workgroups than
 * a launch may have is reported there. */
lbm_status lbm_batch_set_launch(lbm_batch *b, int32_t steps, int32_t block_x, int32_t seg_rows);

/* The batch's launch in use: out[0] = steps per launch, out[1] = block_x,
 * out[2] = seg_rows (the two-step length last chosen or set). */
lbm_status lbm_batch_get_launch(const lbm_batch *b, int32_t out[3]);

/* Free the host batch object (the handles and the workspace are untouched). */
void lbm_batch_destroy(lbm_batch *b);

const char *lbm_status_string(lbm_status s);

/* Text of the last error on this handle ("" if none).  Valid until the next
 * call on the handle. */
const char *lbm_last_error(const lbm_handle *h);

/* Free the host handle.  The workspace stays the caller's; the stream is not
 * synchronised. */
void lbm_destroy(lbm_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
