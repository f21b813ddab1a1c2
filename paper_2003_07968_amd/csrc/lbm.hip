// lbm.hip -- host runtime and C ABI (include/lbm.h) of the D2Q9 force-approach
// pseudopotential lattice Boltzmann library for AMD CDNA4 (gfx950): parameter
// checks, workspace layout, launch shapes, the step loop, batches with graph
// replay, the autotuner and the diagnostics reduction.  The method and the
// kernels are described in lbm_kernels.hpp; each storage mode's kernels are
// instantiated in lbm_inst.hip.
#include "lbm_internal.h"
#include "lbm_probe.h"
#include "lbm_kernels.hpp"

#include <mutex>
#include <vector>

using namespace lbmk;

namespace {

// Batch counters of graph replays (batch_pos in lbm_kernels.hpp): p[0] steps
// and p[1] launches since the table was written.
__global__ void set_counters(long long *p, long long steps, long long launches)
{
    p[0] = steps;
    p[1] = launches;
}
__global__ void bump_counters(long long *p, long long steps, long long launches)
{
    p[0] += steps;
    p[1] += launches;
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
    int device;              // HIP device current at lbm_init
    lbm_status sticky;
    std::string last_error;
};

// ---- Statically allocated scratch (lbm_diagnostics_noalloc) ----
//
// The per-tile partial sums and the reduced values of one diagnostics sweep,
// in a device array of fixed size instead of the workspace: at most
// kNoAllocTiles workgroups (tiles of the single-step sweep), then kDiag
// reduced values.  Every GPU the library runs on holds its own copy until
// the process ends.  Host code never uses the array's name as an address: it
// takes the device address from hipGetSymbolAddress, once per device, with
// that device current.
constexpr int kNoAllocTiles = 16384;
constexpr size_t kScratchDoubles = (size_t)kNoAllocTiles * kDiag + kDiag;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device (null: not yet)

// The device address of this device's scratch array (device `dev` must be
// current).
hipError_t scratch_on_device(int dev, double **out)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

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
    long long ctr_steps, ctr_launches;  // what the device counters hold once the
                                        // work enqueued so far has run
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
constexpr int kBatchRowsMin2 = 2, kBatchRowsMax2 = 48;  // default-length search range

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

// Strip width alignment of the two-step pass: 16 columns in every mode (128
// bytes of FP64, 64 of FP32, 32 of FP16).  The FP16 passes are bound by
// instruction issue, so the lanes a coarser alignment leaves idle cost more
// than stores that share a cache line with the neighbouring strip's: on
// 2048-wide lattices 256-lane workgroups make 9 strips of 240 columns instead
// of 10 of 224.
int strip_align2(int) { return 16; }

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

// Workgroups of the two-step pass one CU runs at once, per 256 threads: FP64
// two (its waves per SIMD), FP32 two (as measured best, though four would
// fit), FP16 four.
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
    if (!make_tiles2(nx, ny, bx, ny, strip_align2(storage), &t0)) return false;
    const long long slots = (long long)slots_per_cu2(storage, bx) * cus;
    const long long per_round = std::max(1ll, slots / t0.nstrips);  // segments per round
    long long nseg = per_round;
    if ((ny + nseg - 1) / nseg > max_rows)  // whole rounds of segments of <= max_rows
        nseg = per_round * ((ny + per_round * max_rows - 1) / (per_round * max_rows));
    if ((ny + nseg - 1) / nseg < min_rows) nseg = (ny + min_rows - 1) / min_rows;
    nseg = std::max(1ll, std::min<long long>(nseg, ny));
    for (int r = (int)((ny + nseg - 1) / nseg);; r = std::min(2 * r, ny)) {
        if (make_tiles2(nx, ny, bx, r, strip_align2(storage), tl)) {
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

// The kernels of the handle's storage mode (each mode's launchers live in a
// translation unit of their own).
SweepArgs sweep_args(const lbm_handle *h, const void *src, void *dst, Fields fo, bool two)
{
    return SweepArgs{src,          dst,    h->c,        two ? h->tiles2 : h->tiles,
                     two ? h->bx2 : h->bx, (long long)h->t, h->err, fo,
                     h->rho_snap,  h->partials, h->stream};
}

template <int MODE>
hipError_t run_sweep(lbm_handle *h, const void *src, void *dst, Fields fo,
                     double *partials = nullptr)
{
    SweepArgs a = sweep_args(h, src, dst, fo, false);
    if (partials) a.partials = partials;
    switch (h->c.storage) {
    case LBM_STORE_F64: return launch_sweep<LBM_STORE_F64>(MODE, a);
    case LBM_STORE_F32_SHIFTED: return launch_sweep<LBM_STORE_F32_SHIFTED>(MODE, a);
    case LBM_STORE_F16_SHIFTED: return launch_sweep<LBM_STORE_F16_SHIFTED>(MODE, a);
    case LBM_STORE_F16_LOCAL: return launch_sweep<LBM_STORE_F16_LOCAL>(MODE, a);
    }
    return hipErrorInvalidValue;
}

// Two time steps, t -> t + 2, in one pass.
hipError_t run_sweep2(lbm_handle *h, const void *src, void *dst)
{
    const SweepArgs a = sweep_args(h, src, dst, Fields{}, true);
    switch (h->c.storage) {
    case LBM_STORE_F64: return launch_sweep2<LBM_STORE_F64>(a);
    case LBM_STORE_F32_SHIFTED: return launch_sweep2<LBM_STORE_F32_SHIFTED>(a);
    case LBM_STORE_F16_SHIFTED: return launch_sweep2<LBM_STORE_F16_SHIFTED>(a);
    case LBM_STORE_F16_LOCAL: return launch_sweep2<LBM_STORE_F16_LOCAL>(a);
    }
    return hipErrorInvalidValue;
}

hipError_t run_init(lbm_handle *h, const double *rho0, const double *ux0, const double *uy0)
{
    switch (h->c.storage) {
    case LBM_STORE_F64:
        return launch_init<LBM_STORE_F64>(h->cur, h->c, rho0, ux0, uy0, h->stream);
    case LBM_STORE_F32_SHIFTED:
        return launch_init<LBM_STORE_F32_SHIFTED>(h->cur, h->c, rho0, ux0, uy0, h->stream);
    case LBM_STORE_F16_SHIFTED:
        return launch_init<LBM_STORE_F16_SHIFTED>(h->cur, h->c, rho0, ux0, uy0, h->stream);
    case LBM_STORE_F16_LOCAL:
        return launch_init<LBM_STORE_F16_LOCAL>(h->cur, h->c, rho0, ux0, uy0, h->stream);
    }
    return hipErrorInvalidValue;
}

hipError_t run_permute(lbm_handle *h, const void *in, void *out, int to_canonical)
{
    switch (h->c.storage) {
    case LBM_STORE_F64:
        return launch_permute<LBM_STORE_F64>(in, out, h->c, to_canonical, h->stream);
    case LBM_STORE_F32_SHIFTED:
        return launch_permute<LBM_STORE_F32_SHIFTED>(in, out, h->c, to_canonical, h->stream);
    case LBM_STORE_F16_SHIFTED:
        return launch_permute<LBM_STORE_F16_SHIFTED>(in, out, h->c, to_canonical, h->stream);
    case LBM_STORE_F16_LOCAL:
        return launch_permute<LBM_STORE_F16_LOCAL>(in, out, h->c, to_canonical, h->stream);
    }
    return hipErrorInvalidValue;
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


BatchArgs batch_args(const lbm_batch *b, bool two, const long long *ctr, long long steps_add,
                     int launches_add)
{
    return BatchArgs{b->d_table,
                     (int)b->members.size(),
                     ctr,
                     steps_add,
                     launches_add,
                     two ? b->bx2 : b->bx,
                     (unsigned)(two ? b->total_tiles2 : b->total_tiles),
                     b->force_on,
                     b->coll,
                     b->stream};
}

// One batched launch of `steps` (1 or 2) steps starting where batch_pos says:
// eager launches pass the position (ctr = nullptr), captured ones their offset
// from the device counters.
hipError_t batch_launch_steps(lbm_batch *b, int steps, const long long *ctr, long long steps_add,
                              int launches_add)
{
    const BatchArgs a = batch_args(b, steps == 2, ctr, steps_add, launches_add);
    if (steps == 2) {
        switch (b->storage) {
        case LBM_STORE_F64: return launch_batch2<LBM_STORE_F64>(a);
        case LBM_STORE_F32_SHIFTED: return launch_batch2<LBM_STORE_F32_SHIFTED>(a);
        case LBM_STORE_F16_SHIFTED: return launch_batch2<LBM_STORE_F16_SHIFTED>(a);
        case LBM_STORE_F16_LOCAL: return launch_batch2<LBM_STORE_F16_LOCAL>(a);
        }
        return hipErrorInvalidValue;
    }
    switch (b->storage) {
    case LBM_STORE_F64: return launch_batch<LBM_STORE_F64>(a);
    case LBM_STORE_F32_SHIFTED: return launch_batch<LBM_STORE_F32_SHIFTED>(a);
    case LBM_STORE_F16_SHIFTED: return launch_batch<LBM_STORE_F16_SHIFTED>(a);
    case LBM_STORE_F16_LOCAL: return launch_batch<LBM_STORE_F16_LOCAL>(a);
    }
    return hipErrorInvalidValue;
}

// Steps per launch of a batch: two unless the caller has asked for single
// steps.
int batch_fuse(const lbm_batch *b) { return b->fuse_max; }

// Average duration in microseconds of `reps` calls of fn on `stream`, after
// `warm` untimed calls.  Returns a negative value on a HIP error.
template <class Fn>
double time_launches(hipStream_t stream, int reps, Fn &&fn, int warm = 1)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.0;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.0;
    }
    double us = -1.0;
    bool warmed = true;
    for (int w = 0; w < warm && warmed; ++w)
        warmed = fn() == hipSuccess;
    if (warmed && hipEventRecord(e0, stream) == hipSuccess) {
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

// A launch shape and its timed duration per launch.
struct Shape {
    double us;
    int bx, rows;
};

// Second pass of a tuner: the kRefine fastest shapes of the first pass (one
// sample of three launches each) timed again as the best of three samples of
// twenty launches, each after five untimed ones (a table upload before it
// leaves the device idle), so that a shape wins by being faster and not by
// one lucky or cold sample.  set(shape) puts a shape in place (false: it does not fit), fn()
// makes one launch.  Returns the fastest shape; us < 0 if a launch failed,
// or 1e300 with no candidates.
constexpr int kRefine = 3;
template <class Set, class Fn>
Shape refine_shapes(hipStream_t stream, std::vector<Shape> cands, Set &&set, Fn &&fn)
{
    std::sort(cands.begin(), cands.end(),
              [](const Shape &a, const Shape &b) { return a.us < b.us; });
    Shape best{1e300, 0, 0};
    for (size_t i = 0; i < cands.size() && i < (size_t)kRefine; ++i) {
        if (!set(cands[i])) continue;
        double t = 1e300;
        for (int k = 0; k < 3; ++k) {
            const double us = time_launches(stream, 20, fn, 5);
            if (us < 0) return Shape{-1.0, cands[i].bx, cands[i].rows};
            t = std::min(t, us);
        }
        if (t < best.us) best = Shape{t, cands[i].bx, cands[i].rows};
    }
    return best;
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
    const int align = strip_align(b->storage), align2 = strip_align2(b->storage);
    const bool two = batch_fuse(b) == 2;
    if (two && b->auto_rows2 && !b->members.empty()) {
        // the segment length that minimises rounds x (rows + 6) over the whole
        // batch, as for one lattice (the longer one on ties); every length
        // from 2 to 48 rows is tried, so that a batch of equal lattices gets
        // the length that fills whole rounds
        const long long slots =
            (long long)slots_per_cu2(b->storage, b->bx2) * b->members[0]->cus;
        long long best = -1;
        for (int r = kBatchRowsMin2; r <= kBatchRowsMax2; ++r) {
            long long tiles = 0;
            bool ok = true;
            for (const lbm_handle *h : b->members) {
                Tiles t;
                if (!make_tiles2(h->p.nx, h->p.ny, b->bx2, std::min(r, h->p.ny), align2, &t)) {
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
            (two && !make_tiles2(h->p.nx, h->p.ny, b->bx2, std::min(b->rows2, h->p.ny), align2,
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
        hipLaunchKernelGGL(set_counters, dim3(1), dim3(1), 0, b->stream, b->d_ctr, 0ll, 0ll);
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
    b->ctr_steps = 0;
    b->ctr_launches = 0;
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

// Capture kGraphSteps batched steps in a graph: launches of batch_fuse(b)
// steps at their offsets from the device counters, then one kernel that
// moves the counters on by the whole graph.  An even number of launches, so
// a replay leaves every lattice's state in the buffer it started from.
hipError_t batch_capture(lbm_batch *b)
{
    hipGraph_t g;
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    const int per = batch_fuse(b), n = kGraphSteps / per;
    for (int k = 0; k < n && le == hipSuccess; ++k)
        le = batch_launch_steps(b, per, b->d_ctr, (long long)k * per, k);
    if (le == hipSuccess) {
        hipLaunchKernelGGL(bump_counters, dim3(1), dim3(1), 0, b->stream, b->d_ctr,
                           (long long)kGraphSteps, (long long)n);
        le = hipGetLastError();
    }
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

// The step kernels' population traffic with none of their arithmetic: nine
// FP64 planes in the population layout copied as one time step pulls them,
// dst_i(x, y) = src_i(x - c_ix, y - c_iy) (periodic), each workgroup walking
// a segment of rows of a 256-column strip in the XCD-aware tile order, with
// non-temporal stores.  Its bandwidth is the ceiling of that access pattern.
__global__ __launch_bounds__(256) void probe_stream9(const double *__restrict__ src,
                                                     double *__restrict__ dst, int nx, int ny,
                                                     size_t plane, size_t pitch, int nstrips,
                                                     int nseg)
{
    const int tile = lbmk::xcd_tile(blockIdx.x, nstrips * nseg);
    const int seg = tile / nstrips, strip = tile - seg * nstrips;
    const int x = strip * 256 + (int)threadIdx.x;
    if (x >= nx) return;  // no barriers below
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int ys = (int)((long long)seg * ny / nseg), ye = (int)((long long)(seg + 1) * ny / nseg);
    for (int y = ys; y < ye; ++y) {
        const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
        const double *r = src + (size_t)y * pitch;
        const double *rm = src + (size_t)ym * pitch;
        const double *rp = src + (size_t)yp * pitch;
        double v[9];
        v[0] = r[x];
        v[1] = r[plane + xm];
        v[2] = rm[2 * plane + x];
        v[3] = r[3 * plane + xp];
        v[4] = rp[4 * plane + x];
        v[5] = rm[5 * plane + xm];
        v[6] = rm[6 * plane + xp];
        v[7] = rp[7 * plane + xp];
        v[8] = rp[8 * plane + xm];
        double *o = dst + (size_t)y * pitch;
#pragma unroll
        for (int i = 0; i < 9; ++i)
            __builtin_nontemporal_store(v[i], o + (size_t)i * plane + x);
    }
}

constexpr size_t kProbePlaneAlign = 16;  // doubles: rows on 128-byte boundaries
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
    if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;
    h->bx2 = kFuseBx;
    h->fuse = default_rows2(params->nx, params->ny, params->storage, h->bx2, h->cus,
                            &h->seg_rows2, &h->tiles2)
                  ? 2
                  : 1;

    const size_t n = (size_t)params->nx * params->ny;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(fill_u64, dim3(1), dim3(1), 0, h->stream, h->err, ~0ull);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = run_init(h, d_rho0, d_ux0, d_uy0);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(copy_plane, dim3(blocks), dim3(256), 0, h->stream, d_rho0,
                           h->rho_snap, n);
        e = hipGetLastError();
    }
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
            hipError_t e = run_sweep2(h, h->cur, h->nxt);
            if (e != hipSuccess) return dev_fail(h, e, "launching the two-step kernel");
            std::swap(h->cur, h->nxt);
            h->t += 2;
        }
    }
    for (; k < nsteps; ++k) {
        hipError_t e = run_sweep<kStep>(h, h->cur, h->nxt, Fields{});
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
    hipError_t e = run_sweep<kMoments>(h, h->cur, nullptr, fo);
    if (e != hipSuccess) return dev_fail(h, e, "launching the moments kernel");
    return read_sticky(h);
}

lbm_status lbm_diagnostics(lbm_handle *h, double out[6])
{
    if (!h || !out) return LBM_ERR_INVALID_ARG;
    hipError_t e = run_sweep<kDiagnostics>(h, h->cur, nullptr, Fields{});
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

lbm_status lbm_diagnostics_noalloc(lbm_handle *h, double out[6])
{
    if (!h || !out) return LBM_ERR_INVALID_ARG;
    if (h->tiles.ntiles > kNoAllocTiles) {
        char buf[200];
        std::snprintf(buf, sizeof buf,
                      "lbm_diagnostics_noalloc: the diagnostics sweep has %d workgroups, more "
                      "than the %d its static scratch holds (a longer seg_rows in "
                      "lbm_set_launch, or lbm_diagnostics, avoids this)",
                      h->tiles.ntiles, kNoAllocTiles);
        h->last_error = buf;
        return LBM_ERR_INVALID_ARG;
    }
    // the handle's device current for the set-up and the launches
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return dev_fail(h, e, "querying the current device");
    if (prev != h->device && (e = hipSetDevice(h->device)) != hipSuccess)
        return dev_fail(h, e, "selecting the handle's device");
    double *s = nullptr;
    e = scratch_on_device(h->device, &s);
    if (e == hipSuccess) e = run_sweep<kDiagnostics>(h, h->cur, nullptr, Fields{}, s);
    if (e == hipSuccess) {
        double *red = s + (size_t)kNoAllocTiles * kDiag;
        hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(256), 0, h->stream, s,
                           h->tiles.ntiles, red);
        e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(out, red, kDiag * sizeof(double), hipMemcpyDeviceToHost,
                               h->stream);
    }
    lbm_status st = e == hipSuccess ? read_sticky(h)
                                    : dev_fail(h, e, "diagnostics with the static scratch");
    if (prev != h->device) (void)hipSetDevice(prev);
    return st;
}

lbm_status lbm_get_populations(lbm_handle *h, double *d_f)
{
    if (!h || !d_f) return LBM_ERR_INVALID_ARG;
    hipError_t e = run_permute(h, h->cur, d_f, 1);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return dev_fail(h, e, "copying populations out");
    return LBM_OK;
}

lbm_status lbm_set_populations(lbm_handle *h, const double *d_f, int64_t t)
{
    if (!h || !d_f || t < 0) return LBM_ERR_INVALID_ARG;
    hipError_t e = run_permute(h, d_f, h->cur, 0);
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
                  : !make_tiles2(h->p.nx, h->p.ny, bx, rows, strip_align2(h->p.storage), &tl)) {
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
        auto set = [&](const Shape &sh) {
            Tiles tl;
            if (!make_tiles(h->p.nx, h->p.ny, sh.bx, sh.rows, align, &tl)) return false;
            h->bx = sh.bx;
            h->seg_rows = sh.rows;
            h->tiles = tl;
            return true;
        };
        auto launch = [&] { return run_sweep<kStep>(h, h->cur, h->nxt, Fields{}); };
        auto fail = [&] {
            h->bx = bx0;
            h->seg_rows = rows0;
            h->tiles = tl0;
            return dev_fail(h, hipGetLastError(), "timing a launch shape");
        };
        std::vector<Shape> cands;
        for (int bx : kTuneWidths)
            for (int rows : kTuneRows) {
                const Shape sh{0.0, bx, std::min(rows, h->p.ny)};
                if (!set(sh)) continue;
                const double us = time_launches(h->stream, 3, launch);
                if (us < 0) return fail();
                cands.push_back(Shape{us, sh.bx, sh.rows});
            }
        const Shape b = refine_shapes(h->stream, cands, set, launch);
        if (b.us < 0) return fail();
        if (b.us < 1e300) {
            best1 = b.us;
            bx1 = b.bx;
            rows1 = b.rows;
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
        auto set = [&](const Shape &sh) {
            Tiles tl;
            if (!make_tiles2(h->p.nx, h->p.ny, sh.bx, sh.rows, strip_align2(h->p.storage), &tl))
                return false;
            h->bx2 = sh.bx;
            h->seg_rows2 = sh.rows;
            h->tiles2 = tl;
            return true;
        };
        auto launch = [&] { return run_sweep2(h, h->cur, h->nxt); };
        auto fail = [&] {
            h->bx2 = bx0;
            h->seg_rows2 = rows0;
            h->tiles2 = tl0;
            return dev_fail(h, hipGetLastError(), "timing a launch shape");
        };
        std::vector<Shape> cands;
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
                }
                const Shape sh{0.0, bx, r};
                if (!set(sh)) continue;
                const double us = time_launches(h->stream, 3, launch);
                if (us < 0) return fail();
                cands.push_back(Shape{us, bx, r});
            }
        const Shape b = refine_shapes(h->stream, cands, set, launch);
        if (b.us < 0) return fail();
        if (b.us < 1e300) {
            best2 = 0.5 * b.us;
            bx2 = b.bx;
            rows2 = b.rows;
        }
        make_tiles2(h->p.nx, h->p.ny, bx2, rows2, strip_align2(h->p.storage), &h->tiles2);
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
    b->ctr_steps = 0;
    b->ctr_launches = 0;
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
        // the replay starts from the device counters: set them where the
        // batch is if eager launches have moved it on since
        const long long s0 = b->steps_since_upload + done, l0 = b->launches_since_upload + launches;
        hipError_t e = hipSuccess;
        if (b->ctr_steps != s0 || b->ctr_launches != l0) {
            hipLaunchKernelGGL(set_counters, dim3(1), dim3(1), 0, b->stream, b->d_ctr, s0, l0);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipGraphLaunch(b->graph, b->stream);
        if (e != hipSuccess) {
            b->last_error = std::string("launching the batch graph: ") + hipGetErrorString(e);
            return LBM_ERR_DEVICE;
        }
        done += kGraphSteps;
        launches += kGraphSteps / per;
        b->ctr_steps = s0 + kGraphSteps;
        b->ctr_launches = l0 + kGraphSteps / per;
    }
    while (done < nsteps) {
        const int k = nsteps - done >= per ? per : 1;
        const hipError_t e =
            batch_launch_steps(b, k, nullptr, b->steps_since_upload + done,
                               (int)((b->launches_since_upload + launches) & 1));
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
    {
        auto set = [&](const Shape &sh) {
            b->bx = sh.bx;
            b->rows = sh.rows;
            return batch_upload(b) == LBM_OK;
        };
        auto launch = [&] { return batch_launch_steps(b, 1, nullptr, 0, 0); };
        std::vector<Shape> cands;
        for (int bx : kTuneWidths)
            for (int rows : kTuneRows) {
                const Shape sh{0.0, bx, rows};
                if (!set(sh)) continue;
                const double us = time_launches(b->stream, 3, launch);
                if (us >= 0) cands.push_back(Shape{us, bx, rows});
            }
        const Shape best = refine_shapes(b->stream, cands, set, launch);
        if (best.us >= 0 && best.us < 1e300) {
            best1 = best.us;
            bx1 = best.bx;
            rows1 = best.rows;
        }
    }
    b->bx = bx1;
    b->rows = rows1;
    double best2 = 1e300;
    int bx2 = b->bx2, rows2 = b->rows2;
    if (try_two) {
        b->fuse_max = 2;
        b->auto_rows2 = false;
        auto set = [&](const Shape &sh) {
            b->bx2 = sh.bx;
            b->rows2 = sh.rows;
            return batch_upload(b) == LBM_OK;
        };
        auto launch = [&] { return batch_launch_steps(b, 2, nullptr, 0, 0); };
        std::vector<Shape> cands;
        for (int bx : kTuneWidths2) {
            // the default length for this width, then the fixed candidates
            b->bx2 = bx;
            b->auto_rows2 = true;
            const bool have_default = batch_upload(b) == LBM_OK;
            b->auto_rows2 = false;
            if (have_default) {
                const double us = time_launches(b->stream, 3, launch);
                if (us >= 0) cands.push_back(Shape{us, bx, b->rows2});
            }
            for (int rows : kBatchRowsCand2) {
                const Shape sh{0.0, bx, rows};
                if (!set(sh)) continue;
                const double us = time_launches(b->stream, 3, launch);
                if (us >= 0) cands.push_back(Shape{us, bx, rows});
            }
        }
        const Shape best = refine_shapes(b->stream, cands, set, launch);
        if (best.us >= 0 && best.us < 1e300) {
            best2 = 0.5 * best.us;
            bx2 = best.bx;
            rows2 = best.rows;
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

lbm_status lbm_batch_set_launch(lbm_batch *b, int32_t steps, int32_t block_x, int32_t seg_rows)
{
    if (!b) return LBM_ERR_INVALID_ARG;
    if (steps == 2) {
        if ((block_x != 128 && block_x != 256 && block_x != 512) || seg_rows < 0) {
            b->last_error = "two-step pass: block_x must be 128, 256 or 512 and seg_rows >= 0";
            return LBM_ERR_INVALID_ARG;
        }
        b->bx2 = block_x;
        b->auto_rows2 = seg_rows == 0;
        if (seg_rows > 0) b->rows2 = seg_rows;
    } else if (steps == 1) {
        if (block_x < 64 || block_x > 512 || block_x % 64 != 0 || seg_rows < 1) {
            b->last_error = "single steps: block_x must be a multiple of 64 in 64..512 and seg_rows >= 1";
            return LBM_ERR_INVALID_ARG;
        }
        b->bx = block_x;
        b->rows = seg_rows;
    } else {
        b->last_error = "steps per launch must be 1 or 2";
        return LBM_ERR_INVALID_ARG;
    }
    b->fuse_max = steps;
    b->table_valid = false;
    if (b->graph_valid) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph_valid = false;
    }
    return LBM_OK;
}

lbm_status lbm_batch_get_launch(const lbm_batch *b, int32_t out[3])
{
    if (!b || !out) return LBM_ERR_INVALID_ARG;
    const bool two = batch_fuse(b) == 2;
    out[0] = batch_fuse(b);
    out[1] = two ? b->bx2 : b->bx;
    out[2] = two ? b->rows2 : b->rows;
    return LBM_OK;
}

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

size_t lbm_probe_stream_bytes(int32_t nx, int32_t ny)
{
    if (nx < 3 || ny < 3) return 0;
    return kQ * round_up((size_t)nx, kProbePlaneAlign) * (size_t)ny * sizeof(double);
}

lbm_status lbm_probe_stream(const double *d_src, double *d_dst, int32_t nx, int32_t ny,
                            int32_t seg_rows, void *hip_stream)
{
    if (!d_src || !d_dst || d_src == d_dst || nx < 3 || ny < 3 || seg_rows < 1)
        return LBM_ERR_INVALID_ARG;
    const size_t plane = round_up((size_t)nx, kProbePlaneAlign);
    const int nstrips = (nx + 255) / 256;
    const int nseg = (ny + seg_rows - 1) / seg_rows;
    if ((long long)nstrips * nseg > kMaxTiles) return LBM_ERR_INVALID_ARG;
    hipLaunchKernelGGL(probe_stream9, dim3(nstrips * nseg), dim3(256), 0,
                       (hipStream_t)hip_stream, d_src, d_dst, nx, ny, plane, kQ * plane, nstrips,
                       nseg);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_ERR_DEVICE;
}

}  // extern "C"

namespace lbm_internal {

lbm_status enqueue_density(lbm_handle *h, double *d_rho)
{
    if (!h || !d_rho) return LBM_ERR_INVALID_ARG;
    Fields fo{d_rho, nullptr, nullptr, nullptr, nullptr, nullptr};
    hipError_t e = run_sweep<kMoments>(h, h->cur, nullptr, fo);
    return e == hipSuccess ? LBM_OK : dev_fail(h, e, "launching the moments kernel");
}

lbm_status enqueue_populations(lbm_handle *h, double *d_f)
{
    if (!h || !d_f) return LBM_ERR_INVALID_ARG;
    hipError_t e = run_permute(h, h->cur, d_f, 1);
    return e == hipSuccess ? LBM_OK : dev_fail(h, e, "copying populations out");
}

}  // namespace lbm_internal
