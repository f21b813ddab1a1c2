// Continuous-batching serving loop over the lattice library (lbm_server.h).
//
// Host-side scheduler: a FIFO queue of submitted jobs, admission by device
// memory footprint into a caller-owned arena (first-fit, arena.h), one batch
// per (storage mode, force switch, collision operator) advanced by the
// batched step, and retirement with the results copied to the caller's host
// buffers.  Every device operation goes through the public C ABI of lbm.h,
// two enqueue-only forms of its output calls (lbm_internal.h) and plain HIP
// copies on the server's stream.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <list>
#include <new>
#include <string>
#include <vector>

#include "arena.h"
#include "lbm.h"
#include "lbm_internal.h"
#include "lbm_server.h"

namespace {

constexpr int kStorages = 4;
// one batch per (storage mode, force switch, collision operator)
constexpr int kBatchKeys = kStorages * 2 * 2;
// Rounds between checks of the resident jobs' sticky errors when no job
// retires (a round that retires jobs checks them anyway).
constexpr int kErrorCheckRounds = 16;

struct Job {
    int64_t id;
    lbm_params p;
    std::vector<double> rho0;
    int64_t nsteps, remaining;
    double *rho_out, *f_out;
    lbm_handle *h = nullptr;
    size_t ws_off = 0, ws_bytes = 0, buf_off = 0, buf_bytes = 0;
    int key = 0;
    int bypassed = 0;
};

size_t cells(const lbm_params &p) { return (size_t)p.nx * (size_t)p.ny; }

int batch_key(const lbm_params &p)
{
    return (p.storage * 2 + (p.force_on ? 1 : 0)) * 2 + (p.collision == LBM_COLL_MRT ? 1 : 0);
}

size_t buffer_bytes(const lbm_params &p, bool want_f) { return (want_f ? 9 : 1) * cells(p) * 8; }

}  // namespace

struct lbm_server {
    lbm_server_config cfg;
    char *arena_base;
    lbm_arena::Arena arena;
    hipStream_t stream;
    lbm_batch *batches[kBatchKeys];
    std::list<Job *> queue;
    std::vector<Job *> resident;
    std::vector<std::pair<int64_t, int32_t>> done;
    int64_t next_id = 0, submitted = 0, completed = 0, rounds = 0, cell_steps = 0;
    size_t table_bytes = 0;  // arena bytes held by the batch tables
    int rounds_since_check = 0;
    bool broken = false;
};

namespace {

void release_job(lbm_server *s, Job *j)
{
    if (j->h) {
        lbm_destroy(j->h);
        j->h = nullptr;
    }
    if (j->ws_bytes) s->arena.release(j->ws_off, j->ws_bytes);
    if (j->buf_bytes) s->arena.release(j->buf_off, j->buf_bytes);
    j->ws_bytes = j->buf_bytes = 0;
}

void finish(lbm_server *s, Job *j, lbm_status st)
{
    release_job(s, j);
    s->done.emplace_back(j->id, (int32_t)st);
    ++s->completed;
    delete j;
}

// Reserve the job's memory; false (nothing held) if the arena cannot fit it now.
bool reserve(lbm_server *s, Job *j)
{
    const size_t ws = lbm_workspace_bytes(&j->p);
    const size_t buf = buffer_bytes(j->p, j->f_out != nullptr);
    size_t a, b;
    if (!s->arena.alloc(ws, &a)) return false;
    if (!s->arena.alloc(buf, &b)) {
        s->arena.release(a, ws);
        return false;
    }
    j->ws_off = a;
    j->ws_bytes = ws;
    j->buf_off = b;
    j->buf_bytes = buf;
    return true;
}

// Create the lattice of an admitted job: stage rho0 in its buffer, lbm_init.
lbm_status start(lbm_server *s, Job *j)
{
    double *d_buf = (double *)(s->arena_base + j->buf_off);
    hipError_t e = hipMemcpyAsync(d_buf, j->rho0.data(), cells(j->p) * 8, hipMemcpyHostToDevice,
                                  s->stream);
    if (e != hipSuccess) return LBM_ERR_DEVICE;
    lbm_status st = lbm_init(&j->p, s->arena_base + j->ws_off, j->ws_bytes, d_buf, nullptr,
                             nullptr, s->stream, &j->h);
    if (st != LBM_OK) return st;
    return lbm_batch_add(s->batches[j->key], j->h);
}

lbm_status admit(lbm_server *s)
{
    Job *blocked = nullptr;  // the first waiting job that did not fit
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        if ((int)s->resident.size() >= s->cfg.max_resident) break;
        Job *j = *it;
        if (blocked && blocked->bypassed >= s->cfg.max_bypass) break;
        if (!reserve(s, j)) {
            if (!blocked) blocked = j;
            ++it;
            continue;
        }
        if (blocked) ++blocked->bypassed;
        it = s->queue.erase(it);
        const lbm_status st = start(s, j);
        if (st == LBM_ERR_DEVICE) {
            release_job(s, j);
            delete j;
            return st;
        }
        if (st != LBM_OK) {
            finish(s, j, st);
            continue;
        }
        s->resident.push_back(j);
    }
    return LBM_OK;
}

lbm_status step_batches(lbm_server *s)
{
    for (int key = 0; key < kBatchKeys; ++key) {
        int64_t n = s->cfg.quantum;
        bool any = false;
        for (Job *j : s->resident)
            if (j->key == key && j->remaining > 0) {
                n = std::min(n, j->remaining);
                any = true;
            }
        if (!any) continue;
        const lbm_status st = lbm_batch_step(s->batches[key], n);
        if (st != LBM_OK) return st;
        for (Job *j : s->resident)
            if (j->key == key) {
                j->remaining -= n;
                s->cell_steps += n * (int64_t)cells(j->p);
            }
    }
    return LBM_OK;
}

// Retire the finished jobs.  The stream is drained once, after which every
// finishing job's sticky error is read; the outputs of those without one
// (density, populations) are then enqueued with their copies to the caller's
// host buffers, and the stream is drained once more.  A round that retires
// many jobs therefore waits twice in all, not once per job and output.
lbm_status retire(lbm_server *s, int32_t *n_retired)
{
    std::vector<Job *> done;
    for (size_t k = 0; k < s->resident.size();) {
        Job *j = s->resident[k];
        if (j->remaining > 0) {
            ++k;
            continue;
        }
        s->resident.erase(s->resident.begin() + (long)k);
        done.push_back(j);
    }
    if (n_retired) *n_retired = (int32_t)done.size();
    if (done.empty()) return LBM_OK;
    bool device_ok = hipStreamSynchronize(s->stream) == hipSuccess;
    std::vector<lbm_status> st(done.size(), LBM_ERR_DEVICE);
    bool copies = false;
    for (size_t k = 0; k < done.size() && device_ok; ++k) {
        Job *j = done[k];
        st[k] = lbm_batch_remove(s->batches[j->key], j->h);
        if (st[k] == LBM_OK) st[k] = lbm_sync(j->h);
        if (st[k] != LBM_OK) continue;
        double *d_buf = (double *)(s->arena_base + j->buf_off);
        const size_t nc = cells(j->p);
        // stream order keeps the density copy ahead of the populations that
        // reuse the buffer
        if (j->rho_out) {
            st[k] = lbm_internal::enqueue_density(j->h, d_buf);
            if (st[k] == LBM_OK &&
                hipMemcpyAsync(j->rho_out, d_buf, nc * 8, hipMemcpyDeviceToHost, s->stream) !=
                    hipSuccess)
                st[k] = LBM_ERR_DEVICE;
        }
        if (st[k] == LBM_OK && j->f_out) {
            st[k] = lbm_internal::enqueue_populations(j->h, d_buf);
            if (st[k] == LBM_OK &&
                hipMemcpyAsync(j->f_out, d_buf, 9 * nc * 8, hipMemcpyDeviceToHost, s->stream) !=
                    hipSuccess)
                st[k] = LBM_ERR_DEVICE;
        }
        copies = true;
        if (st[k] == LBM_ERR_DEVICE) device_ok = false;
    }
    if (copies && hipStreamSynchronize(s->stream) != hipSuccess) {
        device_ok = false;
        for (lbm_status &x : st)
            if (x == LBM_OK) x = LBM_ERR_DEVICE;
    }
    for (size_t k = 0; k < done.size(); ++k) finish(s, done[k], st[k]);
    return device_ok ? LBM_OK : LBM_ERR_DEVICE;
}

// Retire, with their error, the resident jobs whose lattice has left the EOS
// domain (each one's sticky error word, read after the stream has drained),
// so that a failed job stops holding its slot and memory.
lbm_status retire_failed(lbm_server *s, int32_t *n_retired)
{
    int32_t n = 0;
    if (hipStreamSynchronize(s->stream) != hipSuccess) return LBM_ERR_DEVICE;
    for (size_t k = 0; k < s->resident.size();) {
        Job *j = s->resident[k];
        const lbm_status st = lbm_sync(j->h);
        if (st == LBM_OK) {
            ++k;
            continue;
        }
        if (st != LBM_ERR_DOMAIN) return LBM_ERR_DEVICE;
        s->resident.erase(s->resident.begin() + (long)k);
        if (lbm_batch_remove(s->batches[j->key], j->h) != LBM_OK) return LBM_ERR_DEVICE;
        finish(s, j, st);
        ++n;
    }
    if (n_retired) *n_retired = n;
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_server_create(const lbm_server_config *cfg, void *d_arena, size_t arena_bytes,
                             void *hip_stream, lbm_server **out)
{
    if (!out) return LBM_ERR_INVALID_ARG;
    *out = nullptr;
    if (!cfg || cfg->max_resident < 1 || cfg->quantum < 1 || cfg->max_bypass < 0 || !d_arena ||
        ((uintptr_t)d_arena) % lbm_arena::Arena::kAlign != 0 || !hip_stream)
        return LBM_ERR_INVALID_ARG;
    lbm_server *s = new (std::nothrow) lbm_server();
    if (!s) return LBM_ERR_OOM;
    s->cfg = *cfg;
    s->arena_base = (char *)d_arena;
    s->arena.reset(arena_bytes);
    s->stream = (hipStream_t)hip_stream;
    std::memset(s->batches, 0, sizeof(s->batches));
    const size_t tb = lbm_batch_workspace_bytes(cfg->max_resident);
    for (int key = 0; key < kBatchKeys; ++key) {
        size_t off;
        lbm_status st = s->arena.alloc(tb, &off) ? LBM_OK : LBM_ERR_OOM;
        if (st == LBM_OK)
            st = lbm_batch_create(cfg->max_resident, s->arena_base + off, tb, hip_stream,
                                  &s->batches[key]);
        if (st != LBM_OK) {
            lbm_server_destroy(s);
            return st;
        }
        s->table_bytes += lbm_arena::Arena::rounded(tb);
    }
    *out = s;
    return LBM_OK;
}

size_t lbm_server_job_bytes(const lbm_params *p, int32_t want_populations)
{
    if (!p) return 0;
    const size_t ws = lbm_workspace_bytes(p);
    if (ws == 0) return 0;
    return lbm_arena::Arena::rounded(ws) +
           lbm_arena::Arena::rounded(buffer_bytes(*p, want_populations != 0));
}

lbm_status lbm_server_submit(lbm_server *s, const lbm_params *p, const double *h_rho0,
                             int64_t nsteps, double *h_rho_out, double *h_f_out,
                             int64_t *job_id)
{
    if (!s || !p || !h_rho0 || nsteps < 0) return LBM_ERR_INVALID_ARG;
    const size_t need = lbm_server_job_bytes(p, h_f_out != nullptr);
    if (need == 0) return LBM_ERR_INVALID_ARG;
    if (need > s->arena.capacity() - s->table_bytes) return LBM_ERR_OOM;
    Job *j = new (std::nothrow) Job();
    if (!j) return LBM_ERR_OOM;
    j->id = s->next_id++;
    j->p = *p;
    try {
        j->rho0.assign(h_rho0, h_rho0 + cells(*p));
    } catch (...) {
        delete j;
        return LBM_ERR_OOM;
    }
    j->nsteps = j->remaining = nsteps;
    j->rho_out = h_rho_out;
    j->f_out = h_f_out;
    j->key = batch_key(*p);
    s->queue.push_back(j);
    ++s->submitted;
    if (job_id) *job_id = j->id;
    return LBM_OK;
}

lbm_status lbm_server_advance(lbm_server *s, int32_t *n_retired)
{
    if (n_retired) *n_retired = 0;
    if (!s) return LBM_ERR_INVALID_ARG;
    if (s->broken) return LBM_ERR_DEVICE;
    // jobs admitted with nothing left to do (nsteps = 0) leave before the
    // batched step, which advances every member of a batch.  The round returns
    // as soon as its work is enqueued: the stream is waited for only to copy
    // out the results of retiring jobs and, in such rounds and every
    // kErrorCheckRounds rounds, to find jobs that failed, so the host prepares
    // the next rounds while the device runs this one.
    int32_t early = 0, late = 0, failed = 0;
    lbm_status st = admit(s);
    if (st == LBM_OK) st = retire(s, &early);
    if (st == LBM_OK) st = step_batches(s);
    if (st == LBM_OK) st = retire(s, &late);
    if (st == LBM_OK &&
        (early + late > 0 || ++s->rounds_since_check >= kErrorCheckRounds)) {
        st = retire_failed(s, &failed);
        s->rounds_since_check = 0;
    }
    if (n_retired) *n_retired = early + late + failed;
    if (st != LBM_OK) {
        s->broken = true;
        return LBM_ERR_DEVICE;
    }
    ++s->rounds;
    return LBM_OK;
}

int32_t lbm_server_poll(lbm_server *s, int64_t *ids, int32_t *status, int32_t max)
{
    if (!s || max <= 0 || !ids || !status) return 0;
    const int32_t n = (int32_t)std::min<size_t>((size_t)max, s->done.size());
    for (int32_t k = 0; k < n; ++k) {
        ids[k] = s->done[(size_t)k].first;
        status[k] = s->done[(size_t)k].second;
    }
    s->done.erase(s->done.begin(), s->done.begin() + n);
    return n;
}

lbm_status lbm_server_get_stats(const lbm_server *s, lbm_server_stats *out)
{
    if (!s || !out) return LBM_ERR_INVALID_ARG;
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->queued = (int32_t)s->queue.size();
    out->resident = (int32_t)s->resident.size();
    out->rounds = s->rounds;
    out->cell_steps = s->cell_steps;
    out->arena_bytes = s->arena.capacity();
    out->arena_used = s->arena.used();
    out->arena_peak = s->arena.peak();
    return LBM_OK;
}

void lbm_server_destroy(lbm_server *s)
{
    if (!s) return;
    // work still queued on the stream uses the arena; let it finish before the
    // caller may free it
    (void)hipStreamSynchronize(s->stream);
    for (Job *j : s->resident) {
        if (j->h) lbm_destroy(j->h);
        delete j;
    }
    for (Job *j : s->queue)
        delete j;
    for (lbm_batch *b : s->batches)
        if (b) lbm_batch_destroy(b);
    delete s;
}

}  // extern "C"
