/* Serving loop over the D2Q9 pseudopotential lattice library (lbm.h).
 *
 * Continuous batching of independent simulations ("jobs"): each job is one
 * periodic lattice with its own size and parameters (lbm_params), an initial
 * density field and a step count.  Submitted jobs wait in a queue; a
 * scheduling round (lbm_server_advance) admits waiting jobs while their
 * device-memory footprint fits in the server's arena and a resident slot is
 * free, advances every resident lattice by the same number of steps with one
 * batched launch per two steps (lbm_batch_step; one batch per storage mode, force
 * switch and collision operator, each holding a table for max_resident
 * lattices in the arena), and retires the jobs that have reached their step count,
 * copying their results to host memory.  A job's result is bitwise the one it
 * gives when run alone with lbm_init / lbm_step, whatever else was resident.
 *
 * Memory.  All device memory of the jobs (lattice workspace, the density
 * staging / result buffer) and of the batch tables comes from one
 * caller-owned block (the arena), split by a first-fit allocator; a job's
 * footprint is lbm_server_job_bytes.  Nothing is allocated with hipMalloc.
 *
 * Threads.  A server is not thread-safe; call it from one host thread.  All
 * device work goes to the stream given at creation, which must not be the
 * legacy null stream (batched steps are replayed as captured HIP graphs).
 */
#ifndef LBM_SERVER_H
#define LBM_SERVER_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_server lbm_server;

typedef struct {
    int32_t max_resident;   /* most lattices resident at once (>= 1)                    */
    int32_t quantum;        /* most steps per scheduling round (>= 1)                   */
    int32_t max_bypass;     /* admissions allowed to overtake a queue head that does not
                               fit before admission waits for it (>= 0)                 */
} lbm_server_config;

typedef struct {
    int64_t submitted, completed;
    int32_t queued, resident;
    int64_t rounds;          /* scheduling rounds run                                   */
    int64_t cell_steps;      /* lattice-cell updates performed                           */
    size_t arena_bytes, arena_used, arena_peak;
} lbm_server_stats;

/* Create a server.  d_arena (256-byte aligned, arena_bytes long, caller-owned)
 * is the device memory the jobs are admitted into.  hip_stream is a non-null
 * HIP stream.  LBM_ERR_INVALID_ARG on a bad config, a misaligned arena or a
 * null stream. */
lbm_status lbm_server_create(const lbm_server_config *cfg, void *d_arena, size_t arena_bytes,
                             void *hip_stream, lbm_server **out);

/* Device bytes a job with these parameters occupies while resident (its
 * lattice workspace, rounded to 256 bytes, plus an FP64 buffer of 9 nx ny
 * doubles if want_populations, else of nx ny doubles), or 0 if the parameters
 * are invalid. */
size_t lbm_server_job_bytes(const lbm_params *p, int32_t want_populations);

/* Queue a job.  h_rho0: host FP64 [ny][nx] initial density (copied; the
 * caller may reuse it on return).  nsteps >= 0.  h_rho_out (host, ny nx
 * doubles, may be NULL) receives the density at t = nsteps and h_f_out (host,
 * 9 ny nx doubles in the order of lbm_get_populations, may be NULL) the
 * populations; both must stay valid until the job is reported by
 * lbm_server_poll.  *job_id receives an id, increasing from 0.
 * LBM_ERR_INVALID_ARG for invalid parameters or nsteps < 0; LBM_ERR_OOM if
 * the job's footprint exceeds the whole arena (it could never be admitted). */
lbm_status lbm_server_submit(lbm_server *s, const lbm_params *p, const double *h_rho0,
                             int64_t nsteps, double *h_rho_out, double *h_f_out,
                             int64_t *job_id);

/* One scheduling round: admit (queue order; a job that does not fit may be
 * overtaken by later ones, at most max_bypass times), advance every resident
 * lattice by min(quantum, the fewest steps any resident job still needs),
 * retire finished jobs.  The call returns once the round is enqueued on the
 * server's stream; it waits for the stream only in rounds that retire jobs
 * (their results are in host memory on return) and, then and every 16
 * rounds, to check the resident jobs' sticky errors: a job whose lattice has
 * left the EOS domain is retired at that point with LBM_ERR_DOMAIN, without
 * running its remaining steps.  *n_retired (may be NULL) receives the number
 * of jobs retired in this round.  Returns LBM_OK, or LBM_ERR_DEVICE on a HIP
 * error (the server is then unusable). */
lbm_status lbm_server_advance(lbm_server *s, int32_t *n_retired);

/* Move up to max finished jobs out of the server: ids[k] and status[k]
 * (LBM_OK, or the job's sticky error such as LBM_ERR_DOMAIN, in which case its
 * outputs are not written).  Returns the number reported. */
int32_t lbm_server_poll(lbm_server *s, int64_t *ids, int32_t *status, int32_t max);

/* Counters of the server so far. */
lbm_status lbm_server_get_stats(const lbm_server *s, lbm_server_stats *out);

/* Wait for the server's stream, then free the server's host state.  Resident
 * jobs are dropped (their device memory is the arena's, which stays the
 * caller's and may be freed once this returns). */
void lbm_server_destroy(lbm_server *s);

#ifdef __cplusplus
}
#endif

#endif /* LBM_SERVER_H */
