// Host runtime of lattice batches (declared in include/lb.h).
//
// A batch holds many independent D3Q19 lattices ("domains") of different
// extents, relaxation times, obstacles and forces, and advances all of them
// with ONE kernel launch per step: the tiles of every domain form one work
// list, each workgroup looks up its tile's domain in a device table.  The
// step loop is captured in a HIP graph like the single-lattice one.  The
// launch shape (sites per lane, storage block size, grid, tile order) is
// either the default or chosen by timing the candidates on the batch itself
// (an autotuner whose results are kept per process, keyed by the codec and
// the domains' extents).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lb.h"
#include "lb_host.h"
#include "lb_internal.h"

using namespace lbm;

namespace {

constexpr uint64_t kBatchMagic = 0x4c42424154434821ull;  // "LBBATCH!"
constexpr uint64_t kBatchDead = 0xdeadba7cdeadba7cull;
// Requests of at least kBatchGraphMin steps run as one captured graph of the
// whole run (up to kBatchGraphMax steps), kept for the next request of the
// same length: a 500-step request is one graph launch.
constexpr int kBatchGraphMin = 64;
constexpr int kBatchGraphMax = 1024;

// Launch shape of a batch.  variant: 1 / 2 / 3 = 16- / 8- / 4-byte vectors
// per lane and population; seg_bytes: target bytes of one population's rows
// in a storage block; grid_mult: 0 = one workgroup per tile, k > 0 = k x
// (resident workgroups per CU) x CUs workgroups looping over the tiles;
// wg_cap: at most this many resident workgroups per CU (held by dynamic LDS;
// 0 = as many as the registers allow).  The 4-byte kernel fits six or more
// waves per SIMD, and the best step time has been measured at four or five.
struct Shape {
    int variant = 1;
    int seg_bytes = 32768;
    int grid_mult = 0;
    int tile_order = 0;
    int wg_cap = 0;
};

struct Domain {
    int nx = 0, ny = 0, nz = 0;
    double tau = 0, omega = 0;
    double force[3] = {0, 0, 0};
    uint64_t n = 0, nsolid = 0;
    std::vector<uint8_t> host_flags;  // empty: all fluid
    uint8_t *flags = nullptr;         // device copy (n bytes, zeros when all fluid)
    uint32_t *nbmask = nullptr;       // device, rows x pitch
    uint8_t *rowdirty = nullptr;      // device, rows
    uint32_t *rowcum = nullptr;       // device, rows + 1 (dirty rows before each row)
    Layout lay{};
    uint64_t arr_elems = 0;           // elements of one population array
    void *buf[2] = {nullptr, nullptr};
    int nslots = 0, tile_begin = 0, ntiles = 0;
    int lds_edges = 0, lg_row_lanes = 0;
};

std::mutex g_tune_mu;
std::map<std::string, Shape> g_tuned;  // autotuner results of this process

}  // namespace

struct lb_batch {
    uint64_t magic = 0;
    int count = 0, codec = 0, esize = 4;
    std::vector<Domain> dom;
    Shape shape;
    bool tuned = false;
    void *pool = nullptr;  // both arrays of every domain
    size_t pool_bytes = 0;
    DomDesc *d_doms = nullptr;
    int *d_tile_dom = nullptr;
    double *partials = nullptr;
    unsigned int *ticket = nullptr;
    double *ring = nullptr;
    unsigned long long *counter = nullptr;
    int ntiles = 0, grid = 0, cus = 0;
    size_t lds_pad = 0;  // dynamic LDS per workgroup of the step launch (the shape's wg_cap)
    int cur = 0;
    long long steps = 0;
    hipStream_t stream = nullptr;  // borrowed (NULL: the default stream)
    RunGraphs graphs;
};

namespace {

int check(const lb_batch *b)
{
    if (!b || b->magic != kBatchMagic) return fail(LB_ESTATE, "invalid or destroyed batch handle");
    return LB_OK;
}

int check_dom(const lb_batch *b, int d)
{
    if (int rc = check(b)) return rc;
    if (d < 0 || d >= b->count) return fail(LB_EINVAL, "domain %d out of range [0, %d)", d, b->count);
    return LB_OK;
}

template <class T>
void free_dev(T *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

// Free everything that depends on the launch shape.
void release_shape(lb_batch *b)
{
    b->graphs.invalidate();
    free_dev(b->pool);
    free_dev(b->d_doms);
    free_dev(b->d_tile_dom);
    free_dev(b->partials);
    for (Domain &d : b->dom) {
        free_dev(d.nbmask);
        free_dev(d.rowdirty);
        free_dev(d.rowcum);
        d.buf[0] = d.buf[1] = nullptr;
    }
}

void release_all(lb_batch *b)
{
    release_shape(b);
    for (Domain &d : b->dom) free_dev(d.flags);
    free_dev(b->ticket);
    free_dev(b->ring);
    free_dev(b->counter);
    b->graphs.release();
    b->stream = nullptr;  // borrowed
}

StepArgs domain_args(const lb_batch *b, const Domain &d)
{
    StepArgs a{};
    a.lay = d.lay;
    a.nx = d.nx;
    a.ny = d.ny;
    a.nz = d.nz;
    a.nslots = d.nslots;
    a.lds_edges = d.lds_edges;
    a.lg_row_lanes = d.lg_row_lanes;
    a.tile_order = 0;
    a.div_pitch = make_fastdiv(d.lay.pitch);
    a.div_ny = make_fastdiv((uint32_t)d.ny);
    a.coll = make_coll((float)d.omega, (float)d.force[0], (float)d.force[1], (float)d.force[2]);
    a.nbmask = d.nbmask;
    a.rowdirty = d.rowdirty;
    a.rowcum = d.rowcum;
    return a;
}

// Write the device domain table (the stream is synchronised first: the table
// may be in use by enqueued steps).
int upload_table(lb_batch *b)
{
    std::vector<DomDesc> t(b->count);
    for (int k = 0; k < b->count; ++k) {
        const Domain &d = b->dom[k];
        t[k].s = domain_args(b, d);
        t[k].buf[0] = d.buf[0];
        t[k].buf[1] = d.buf[1];
        t[k].tile_begin = d.tile_begin;
        t[k].ntiles = d.ntiles;
        t[k].n_fluid = (double)(d.n - d.nsolid);
    }
    HIP_OR_FAIL(hipStreamSynchronize(b->stream));
    HIP_OR_FAIL(hipMemcpy(b->d_doms, t.data(), t.size() * sizeof(DomDesc), hipMemcpyHostToDevice));
    return LB_OK;
}

// Lay out every domain for shape s, allocate the arrays (zeroed), masks and
// tables.  Any previous state is discarded.
int configure(lb_batch *b, const Shape &s)
{
    release_shape(b);
    b->shape = s;
    const int V = sites_per_thread(b->codec, s.variant);
    const int es = b->esize;
    uint64_t pool_elems = 0;
    int tiles = 0;
    std::vector<uint64_t> start(b->count);
    for (int k = 0; k < b->count; ++k) {
        Domain &d = b->dom[k];
        const uint32_t pitch = (uint32_t)((d.nx + V - 1) / V * V);
        const uint64_t rows = (uint64_t)d.ny * d.nz;
        uint64_t R = 1;
        while ((R * 2) * pitch * es <= (uint64_t)s.seg_bytes && R < rows) R *= 2;
        uint32_t lg = 0;
        while ((1ull << lg) < R) ++lg;
        d.lay.nx = (uint32_t)d.nx;
        d.lay.pitch = pitch;
        d.lay.lg_r = lg;
        if (!block_fits(R * pitch, kQ, es)) return fail(LB_EINVAL, "domain %d: rows of %u elements are too long", k, pitch);
        d.lay.seg = (uint32_t)(R * pitch);
        d.lay.blk = (uint32_t)(kQ * R * pitch);
        d.arr_elems = (rows + R - 1) / R * d.lay.blk;
        const uint64_t slots = rows * pitch / V;
        if (slots > 0x7fffffffull) return fail(LB_EINVAL, "domain %d is too large for a batch", k);
        d.nslots = (int)slots;
        d.ntiles = (int)((slots + kBlock - 1) / kBlock);
        d.tile_begin = tiles;
        if ((int64_t)tiles + d.ntiles > 0x7fffffffll) return fail(LB_EINVAL, "too many tiles in the batch");
        tiles += d.ntiles;
        const int row_lanes = (int)(pitch / V);
        d.lds_edges = 1;  // x-edge elements held in the same tile pass through LDS
        d.lg_row_lanes = 0;
        while ((1 << d.lg_row_lanes) < row_lanes) ++d.lg_row_lanes;
        // both arrays of the domain, each starting on a 256-byte boundary
        const uint64_t align = 256 / es;
        start[k] = pool_elems;
        pool_elems += 2 * ((d.arr_elems + align - 1) / align * align);
    }
    b->ntiles = tiles;
    b->pool_bytes = (size_t)pool_elems * es;
    hipError_t e = hipMalloc(&b->pool, b->pool_bytes);
    if (e != hipSuccess) return fail(LB_ENOMEM, "hipMalloc(%zu bytes of populations): %s", b->pool_bytes, hipGetErrorString(e));
    HIP_OR_FAIL(hipMemsetAsync(b->pool, 0, b->pool_bytes, b->stream));
    std::vector<int> tile_dom(tiles);
    for (int k = 0; k < b->count; ++k) {
        Domain &d = b->dom[k];
        const uint64_t align = 256 / es;
        const uint64_t stride = (d.arr_elems + align - 1) / align * align;
        d.buf[0] = static_cast<char *>(b->pool) + start[k] * es;
        d.buf[1] = static_cast<char *>(b->pool) + (start[k] + stride) * es;
        const uint64_t rows = (uint64_t)d.ny * d.nz;
        e = hipMalloc(&d.nbmask, rows * d.lay.pitch * sizeof(uint32_t) + 64);
        if (e != hipSuccess) return fail(LB_ENOMEM, "hipMalloc(masks): %s", hipGetErrorString(e));
        e = hipMalloc(&d.rowdirty, rows);
        if (e != hipSuccess) return fail(LB_ENOMEM, "hipMalloc(rows): %s", hipGetErrorString(e));
        e = hipMalloc(&d.rowcum, (rows + 1) * sizeof(uint32_t));
        if (e != hipSuccess) return fail(LB_ENOMEM, "hipMalloc(rows): %s", hipGetErrorString(e));
        HIP_OR_FAIL(launch_masks(d.flags, d.nx, d.ny, d.nz, (int)d.lay.pitch, d.nbmask, d.rowdirty, d.rowcum,
                                 b->stream));
        std::fill(tile_dom.begin() + d.tile_begin, tile_dom.begin() + d.tile_begin + d.ntiles, k);
    }
    e = hipMalloc(&b->d_doms, (size_t)b->count * sizeof(DomDesc));
    if (e != hipSuccess) return fail(LB_ENOMEM, "hipMalloc(domain table): %s", hipGetErrorString(e));
    e = hipMalloc(&b->d_tile_dom, (size_t)tiles * sizeof(int));
    if (e != hipSuccess) return fail(LB_ENOMEM, "hipMalloc(tile list): %s", hipGetErrorString(e));
    e = hipMalloc(&b->partials, (size_t)tiles * 8 * sizeof(double));  // two buffers, for runs of steps
    if (e != hipSuccess) return fail(LB_ENOMEM, "hipMalloc(partials): %s", hipGetErrorString(e));
    HIP_OR_FAIL(hipStreamSynchronize(b->stream));
    HIP_OR_FAIL(hipMemcpy(b->d_tile_dom, tile_dom.data(), tile_dom.size() * sizeof(int), hipMemcpyHostToDevice));
    if (int rc = upload_table(b)) return rc;
    b->lds_pad = batch_cap_lds(b->codec, s.variant, s.wg_cap);
    const int occ = batch_occupancy(b->codec, s.variant, b->lds_pad);
    int64_t grid = tiles;
    if (s.grid_mult > 0) grid = std::min<int64_t>(grid, (int64_t)s.grid_mult * occ * b->cus);
    b->grid = (int)std::max<int64_t>(grid, 1);
    b->cur = 0;
    return LB_OK;
}

// Totals of the batch step whose tile partials are in buffer buf (0 or 1).
BatchTotalsArgs batch_totals_args(const lb_batch *b, int buf)
{
    BatchTotalsArgs t{};
    t.doms = b->d_doms;
    t.ndoms = b->count;
    t.partials = b->partials + (size_t)buf * 4 * b->ntiles;
    t.ticket = b->ticket;
    t.ring = b->ring;
    t.step_counter = b->counter;
    return t;
}

// count >= 1 steps from buf[parity] as one run: step k writes its tile
// partials into buffer k & 1, the first workgroup of step k + 1 appends the
// per-domain totals of step k, and one totals kernel closes the run (the
// rings hold the same values as with one totals kernel per step).
int enqueue_run(lb_batch *b, int parity, int count, hipStream_t s)
{
    for (int k = 0; k < count; ++k) {
        BatchArgs a{};
        a.doms = b->d_doms;
        a.tile_dom = b->d_tile_dom;
        a.ntiles = b->ntiles;
        a.parity = parity ^ (k & 1);
        a.tile_order = b->shape.tile_order;
        a.partials = b->partials + (size_t)(k & 1) * 4 * b->ntiles;
        if (k > 0) a.prev = batch_totals_args(b, (k - 1) & 1);
        HIP_OR_FAIL(launch_batch_step(b->codec, b->shape.variant, a, b->grid, b->lds_pad, s));
    }
    HIP_OR_FAIL(launch_batch_totals(batch_totals_args(b, (count - 1) & 1), s));
    return LB_OK;
}

// Capture the run of len steps from parity unless it is held already (a new
// length, or a changed launch shape or argument, drops the held graphs).
int ensure_graph(lb_batch *b, int len, int parity)
{
    RunGraphs &G = b->graphs;
    if (G.len != len) G.invalidate();
    if (G.exec[parity]) return LB_OK;
    if (!G.cap) HIP_OR_FAIL(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
    HIP_OR_FAIL(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_run(b, parity, len, G.cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(G.cap, &g);
    if (rc != LB_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(LB_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&G.exec[parity], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        G.exec[parity] = nullptr;
        return fail(LB_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    G.len = len;
    return LB_OK;
}

// Capture the graphs enqueue_steps(b, n) will replay, without launching them.
int prepare_graphs(lb_batch *b, int n)
{
    if (n < kBatchGraphMin) return LB_OK;
    const int len = std::min(n, kBatchGraphMax);
    if (int rc = ensure_graph(b, len, b->cur)) return rc;
    if ((len & 1) && n >= 2 * len) return ensure_graph(b, len, b->cur ^ 1);
    return LB_OK;
}

int enqueue_steps(lb_batch *b, int n)
{
    int plain = n;
    if (plain >= kBatchGraphMin) {
        const int len = std::min(plain, kBatchGraphMax);
        while (plain >= len) {
            if (int rc = ensure_graph(b, len, b->cur)) return rc;
            HIP_OR_FAIL(hipGraphLaunch(b->graphs.exec[b->cur], b->stream));
            b->cur ^= len & 1;
            b->steps += len;
            plain -= len;
        }
    }
    if (plain > 0) {
        if (int rc = enqueue_run(b, b->cur, plain, b->stream)) return rc;
        b->cur ^= plain & 1;
        b->steps += plain;
    }
    return LB_OK;
}

// Mean milliseconds per step of `n` steps (after `warm` untimed ones).
int time_steps(lb_batch *b, int warm, int n, double *ms)
{
    if (int rc = enqueue_steps(b, warm)) return rc;
    if (int rc = prepare_graphs(b, n)) return rc;
    Events evs(2);
    HIP_OR_FAIL(evs.create());
    hipEvent_t e0 = evs[0], e1 = evs[1];
    int rc = LB_OK;
    if (hipEventRecord(e0, b->stream) != hipSuccess) rc = fail(LB_EHIP, "hipEventRecord");
    if (rc == LB_OK) rc = enqueue_steps(b, n);
    if (rc == LB_OK && hipEventRecord(e1, b->stream) != hipSuccess) rc = fail(LB_EHIP, "hipEventRecord");
    float t = 0.0f;
    if (rc == LB_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(LB_EHIP, "hipEventSynchronize");
    if (rc == LB_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = fail(LB_EHIP, "hipEventElapsedTime");
    if (rc == LB_OK) *ms = n > 0 ? (double)t / n : 0.0;
    return rc;
}

std::string tune_key(const lb_batch *b)
{
    std::vector<std::string> parts;
    for (const Domain &d : b->dom) {
        char buf[64];
        snprintf(buf, sizeof buf, "%dx%dx%d%s", d.nx, d.ny, d.nz, d.nsolid ? "s" : "");
        parts.push_back(buf);
    }
    std::sort(parts.begin(), parts.end());
    std::string key = std::to_string(b->codec);
    for (const std::string &p : parts) key += "," + p;
    return key;
}

// Time every candidate shape on the batch (best of two timings of 24 steps;
// its state is discarded) and keep the fastest.
int autotune(lb_batch *b)
{
    const std::string key = tune_key(b);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            b->tuned = true;
            return configure(b, it->second);
        }
    }
    Shape best;
    double best_ms = 1e300;
    const int seg_opts[] = {32768, 4096};
    const int grid_opts[] = {0, 1, 2};
    for (int variant = 1; variant <= 3; ++variant) {
        for (int seg : seg_opts) {
            Shape s;
            s.variant = variant;
            s.seg_bytes = seg;
            if (int rc = configure(b, s)) return rc;
            for (int gm : grid_opts) {
                // workgroup caps: for the 4-byte kernel with one workgroup per tile
                const int ncaps = (variant == 3 && gm == 0) ? 3 : 1;
                for (int ci = 0; ci < ncaps; ++ci) {
                for (int order = 0; order < 2; ++order) {
                    s.grid_mult = gm;
                    s.tile_order = order;
                    s.wg_cap = ci == 0 ? 0 : 3 + ci;  // none, 4, 5
                    b->lds_pad = batch_cap_lds(b->codec, variant, s.wg_cap);
                    const int occ = batch_occupancy(b->codec, variant, b->lds_pad);
                    int64_t grid = b->ntiles;
                    if (gm > 0) grid = std::min<int64_t>(grid, (int64_t)gm * occ * b->cus);
                    b->grid = (int)std::max<int64_t>(grid, 1);
                    b->shape = s;
                    b->graphs.invalidate();
                    double ms = 1e300;
                    for (int rep = 0; rep < 2; ++rep) {  // best of two timings of 24 steps
                        double t = 0;
                        if (int rc = time_steps(b, rep == 0 ? 4 : 0, 24, &t)) return rc;
                        ms = std::min(ms, t);
                    }
                    if (ms < best_ms) {
                        best_ms = ms;
                        best = s;
                    }
                }
                }
            }
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[key] = best;
    }
    b->tuned = true;
    return configure(b, best);
}

}  // namespace

extern "C" {

lb_batch *lb_batch_create(int count, const int *dims, const double *taus, const uint8_t *const *flags, int storage,
                          void *hip_stream, int autotune_shape)
{
    if (count < 1 || !dims || !taus) {
        fail(LB_EINVAL, "a batch needs count >= 1, dims and taus");
        return nullptr;
    }
    if (storage != LB_F32 && storage != LB_F16S && storage != LB_BF16S) {
        fail(LB_EINVAL, "storage codec %d is not available in batches (LB_F32, LB_F16S, LB_BF16S)", storage);
        return nullptr;
    }
    for (int k = 0; k < count; ++k) {
        const int nx = dims[3 * k], ny = dims[3 * k + 1], nz = dims[3 * k + 2];
        if (nx < 1 || ny < 1 || nz < 1) {
            fail(LB_EINVAL, "domain %d: extents must be >= 1 (got %d x %d x %d)", k, nx, ny, nz);
            return nullptr;
        }
        if ((uint64_t)nx * ny * nz > 0x7fffffffull - 4096 || nx > 65536) {
            fail(LB_EINVAL, "domain %d is too large for a batch", k);
            return nullptr;
        }
        if (!(taus[k] > 0.5)) {
            fail(LB_EINVAL, "domain %d: tau must be > 0.5 or +inf (got %g)", k, taus[k]);
            return nullptr;
        }
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        fail(LB_EHIP, "no HIP device available");
        return nullptr;
    }
    lb_batch *b = new (std::nothrow) lb_batch();
    if (!b) {
        fail(LB_ENOMEM, "host allocation failed");
        return nullptr;
    }
    b->count = count;
    b->codec = storage == LB_F32 ? kF32 : (storage == LB_F16S ? kF16 : kBF16);
    b->esize = storage == LB_F32 ? 4 : 2;
    b->dom.resize(count);
    auto bail = [&](int code, const char *what, hipError_t e) -> lb_batch * {
        release_all(b);
        delete b;
        fail(code, "%s: %s", what, hipGetErrorString(e));
        return nullptr;
    };
    hipError_t e;
    b->stream = static_cast<hipStream_t>(hip_stream);  // NULL: the default stream (as lb_create_ex)
    int dev = 0;
    hipDeviceProp_t prop;
    if ((e = hipGetDevice(&dev)) != hipSuccess || (e = hipGetDeviceProperties(&prop, dev)) != hipSuccess)
        return bail(LB_EHIP, "device query", e);
    b->cus = prop.multiProcessorCount;
    for (int k = 0; k < count; ++k) {
        Domain &d = b->dom[k];
        d.nx = dims[3 * k];
        d.ny = dims[3 * k + 1];
        d.nz = dims[3 * k + 2];
        d.tau = taus[k];
        d.omega = std::isinf(taus[k]) ? 0.0 : 1.0 / taus[k];
        d.n = (uint64_t)d.nx * d.ny * d.nz;
        const uint8_t *f = flags ? flags[k] : nullptr;
        if (f) {
            for (uint64_t s = 0; s < d.n; ++s) {
                if (f[s] > 1) {
                    release_all(b);
                    delete b;
                    fail(LB_EINVAL, "domain %d: flag value %d at site %llu (allowed: 0 fluid, 1 solid)", k, (int)f[s],
                         (unsigned long long)s);
                    return nullptr;
                }
                d.nsolid += f[s];
            }
            d.host_flags.assign(f, f + d.n);
        }
        if ((e = hipMalloc(&d.flags, d.n)) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc(flags)", e);
        if (f)
            e = hipMemcpy(d.flags, f, d.n, hipMemcpyHostToDevice);
        else
            e = hipMemset(d.flags, 0, d.n);
        if (e != hipSuccess) return bail(LB_EHIP, "flags upload", e);
    }
    if ((e = hipMalloc(&b->ticket, sizeof(unsigned int))) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc", e);
    if ((e = hipMalloc(&b->counter, sizeof(unsigned long long))) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc", e);
    if ((e = hipMalloc(&b->ring, (size_t)count * kRingCap * 4 * sizeof(double))) != hipSuccess)
        return bail(LB_ENOMEM, "hipMalloc(ring)", e);
    (void)hipMemset(b->ticket, 0, sizeof(unsigned int));
    (void)hipMemset(b->counter, 0, sizeof(unsigned long long));
    (void)hipMemset(b->ring, 0, (size_t)count * kRingCap * 4 * sizeof(double));

    b->magic = kBatchMagic;
    Shape s;
    s.variant = (int)env_long("LB_BATCH_KERNEL", 1);
    s.seg_bytes = (int)env_long("LB_BATCH_SEG_BYTES", 32768);
    s.grid_mult = (int)env_long("LB_BATCH_GRID", 0);
    s.tile_order = (int)env_long("LB_BATCH_TILE_ORDER", 0);
    s.wg_cap = (int)env_long("LB_BATCH_WG_CAP", 0);
    if (s.variant < 1 || s.variant > 3 || s.seg_bytes < 64 || s.grid_mult < 0 || s.wg_cap < 0 || (s.wg_cap > 0 && s.wg_cap < 3) ||
        s.tile_order < 0 || s.tile_order > 2) {
        release_all(b);
        delete b;
        fail(LB_EINVAL, "invalid LB_BATCH_* setting");
        return nullptr;
    }
    int rc = autotune_shape ? autotune(b) : configure(b, s);
    if (rc == LB_OK && hipMemset(b->counter, 0, sizeof(unsigned long long)) != hipSuccess) rc = fail(LB_EHIP, "hipMemset");
    if (rc == LB_OK && hipStreamSynchronize(b->stream) != hipSuccess) rc = fail(LB_EHIP, "hipStreamSynchronize");
    if (rc != LB_OK) {
        const std::string msg = lb_last_error();
        release_all(b);
        b->magic = kBatchDead;
        delete b;
        fail(rc, "%s", msg.c_str());
        return nullptr;
    }
    b->steps = 0;
    return b;
}

void lb_batch_destroy(lb_batch *b)
{
    if (!b || b->magic != kBatchMagic) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    release_all(b);
    b->magic = kBatchDead;
    delete b;
}

int lb_batch_set_force(lb_batch *b, int d, double fx, double fy, double fz)
{
    if (int rc = check(b)) return rc;
    if (d < -1 || d >= b->count) return fail(LB_EINVAL, "domain %d out of range", d);
    if (!std::isfinite(fx) || !std::isfinite(fy) || !std::isfinite(fz)) return fail(LB_EINVAL, "force must be finite");
    for (int k = 0; k < b->count; ++k) {
        if (d >= 0 && k != d) continue;
        b->dom[k].force[0] = fx;
        b->dom[k].force[1] = fy;
        b->dom[k].force[2] = fz;
    }
    return upload_table(b);
}

int lb_batch_init_eq(lb_batch *b, int d, const double *rho, const double *u)
{
    if (int rc = check_dom(b, d)) return rc;
    const Domain &dm = b->dom[d];
    InitArgs a{};
    a.dst = dm.buf[b->cur];
    a.lay = dm.lay;
    a.n = (int)dm.n;
    a.rho = rho;
    a.u = u;
    a.flags = dm.flags;
    HIP_OR_FAIL(launch_init(b->codec, a, b->stream));
    return LB_OK;
}

int lb_batch_step(lb_batch *b, int n)
{
    if (int rc = check(b)) return rc;
    if (n < 0) return fail(LB_EINVAL, "n must be >= 0");
    return enqueue_steps(b, n);
}

int lb_batch_macros(lb_batch *b, int d, float *rho, float *u)
{
    if (int rc = check_dom(b, d)) return rc;
    if (!rho && !u) return LB_OK;
    const Domain &dm = b->dom[d];
    MacroArgs a{};
    a.src = dm.buf[b->cur];
    a.lay = dm.lay;
    a.n = (int)dm.n;
    a.fx = (float)dm.force[0];
    a.fy = (float)dm.force[1];
    a.fz = (float)dm.force[2];
    a.flags = dm.flags;
    a.rho = rho;
    a.u = u;
    HIP_OR_FAIL(launch_macros(b->codec, a, b->stream));
    return LB_OK;
}

int lb_batch_sums(lb_batch *b, int d, double *out, int k)
{
    if (int rc = check_dom(b, d)) return rc;
    if (k < 1 || k > kRingCap) return fail(LB_EINVAL, "k must be in [1, %d]", kRingCap);
    if (!out) return fail(LB_EINVAL, "NULL output");
    if (b->steps < k) return fail(LB_EINVAL, "only %lld steps done", b->steps);
    HIP_OR_FAIL(hipStreamSynchronize(b->stream));
    unsigned long long done = 0;
    HIP_OR_FAIL(hipMemcpy(&done, b->counter, sizeof done, hipMemcpyDeviceToHost));
    std::vector<double> ring((size_t)kRingCap * 4);
    HIP_OR_FAIL(hipMemcpy(ring.data(), b->ring + (size_t)d * kRingCap * 4, ring.size() * sizeof(double),
                          hipMemcpyDeviceToHost));
    bool bad = false;
    for (int j = 0; j < k; ++j) {
        const unsigned long long step = done - (unsigned long long)k + j;
        for (int c = 0; c < 4; ++c) {
            out[4 * j + c] = ring[4 * (step % kRingCap) + c];
            if (!std::isfinite(out[4 * j + c])) bad = true;
        }
    }
    if (bad) return fail(LB_EUNSTABLE, "domain %d: non-finite mass or momentum total", d);
    return LB_OK;
}

static int batch_copy_f(lb_batch *b, int d, void *ptr, size_t bytes, int where, bool to_lattice)
{
    if (int rc = check_dom(b, d)) return rc;
    const Domain &dm = b->dom[d];
    const size_t want = (size_t)kQ * dm.n * b->esize;
    if (bytes != want) return fail(LB_EINVAL, "buffer is %zu bytes, expected %zu", bytes, want);
    if (!ptr) return fail(LB_EINVAL, "NULL buffer");
    if (where != LB_HOST && where != LB_DEVICE) return fail(LB_EINVAL, "where must be LB_HOST or LB_DEVICE");
    void *planes = ptr;
    if (where == LB_HOST) {
        hipError_t e = hipMalloc(&planes, bytes);
        if (e != hipSuccess) return fail(LB_ENOMEM, "hipMalloc(staging): %s", hipGetErrorString(e));
        if (to_lattice && (e = hipMemcpyAsync(planes, ptr, bytes, hipMemcpyHostToDevice, b->stream)) != hipSuccess) {
            (void)hipFree(planes);
            return fail(LB_EHIP, "hipMemcpyAsync: %s", hipGetErrorString(e));
        }
    }
    hipError_t e = launch_repack(planes, dm.buf[b->cur], dm.lay, (int64_t)dm.n, b->esize, to_lattice, b->stream);
    if (e == hipSuccess && where == LB_HOST && !to_lattice)
        e = hipMemcpyAsync(ptr, planes, bytes, hipMemcpyDeviceToHost, b->stream);
    if (where == LB_HOST) {
        const hipError_t s = hipStreamSynchronize(b->stream);
        (void)hipFree(planes);
        if (e == hipSuccess) e = s;
    }
    if (e != hipSuccess) return fail(LB_EHIP, "population copy: %s", hipGetErrorString(e));
    return LB_OK;
}

int lb_batch_get_f(lb_batch *b, int d, void *buf, size_t bytes, int where)
{
    return batch_copy_f(b, d, buf, bytes, where, false);
}

int lb_batch_set_f(lb_batch *b, int d, const void *buf, size_t bytes, int where)
{
    return batch_copy_f(b, d, const_cast<void *>(buf), bytes, where, true);
}

int lb_batch_sync(lb_batch *b)
{
    if (int rc = check(b)) return rc;
    HIP_OR_FAIL(hipStreamSynchronize(b->stream));
    return LB_OK;
}

long long lb_batch_steps_done(lb_batch *b)
{
    if (check(b)) return -1;
    return b->steps;
}

long long lb_batch_query(lb_batch *b, int key)
{
    if (check(b)) return -1;
    long long v = 0;
    switch (key) {
        case 0: return b->shape.variant;
        case 1: return sites_per_thread(b->codec, b->shape.variant);
        case 2: return b->grid;
        case 3: return b->ntiles;
        case 4: return b->shape.tile_order;
        case 5: return b->count;
        case 6:
            for (const Domain &d : b->dom) v += (long long)d.n;
            return v;
        case 7:
            for (const Domain &d : b->dom) v += (long long)(d.n - d.nsolid);
            return v;
        case 8: return (long long)b->pool_bytes;
        case 9: return b->shape.seg_bytes;
        case 10: return b->shape.grid_mult;
        case 11: return b->tuned ? 1 : 0;
        case 12: return b->shape.wg_cap;
        default: fail(LB_EINVAL, "unknown query key %d", key); return -1;
    }
}

int lb_batch_time_steps(lb_batch *b, int n, double *ms)
{
    if (int rc = check(b)) return rc;
    if (n < 1 || !ms) return fail(LB_EINVAL, "n >= 1 and a result pointer are required");
    return time_steps(b, 0, n, ms);
}

int lb_batch_time_step_kernel(lb_batch *b, int n, double *ms)
{
    if (int rc = check(b)) return rc;
    if (n < 1 || !ms) return fail(LB_EINVAL, "n >= 1 and a result pointer are required");
    Events ev(2 * (size_t)n);
    HIP_OR_FAIL(ev.create());
    int rc = LB_OK;
    for (int k = 0; k < n && rc == LB_OK; ++k) {
        BatchArgs a{};
        a.doms = b->d_doms;
        a.tile_dom = b->d_tile_dom;
        a.ntiles = b->ntiles;
        a.parity = b->cur;
        a.tile_order = b->shape.tile_order;
        a.partials = b->partials;
        if (hipEventRecord(ev[2 * k], b->stream) != hipSuccess) rc = fail(LB_EHIP, "hipEventRecord");
        if (rc == LB_OK && launch_batch_step(b->codec, b->shape.variant, a, b->grid, b->lds_pad, b->stream) != hipSuccess)
            rc = fail(LB_EHIP, "batch step launch");
        if (rc == LB_OK && hipEventRecord(ev[2 * k + 1], b->stream) != hipSuccess) rc = fail(LB_EHIP, "hipEventRecord");
        if (rc == LB_OK) {
            BatchTotalsArgs t{};
            t.doms = b->d_doms;
            t.ndoms = b->count;
            t.partials = b->partials;
            t.ticket = b->ticket;
            t.ring = b->ring;
            t.step_counter = b->counter;
            if (launch_batch_totals(t, b->stream) != hipSuccess) rc = fail(LB_EHIP, "batch totals launch");
        }
        if (rc == LB_OK) {
            b->cur ^= 1;
            b->steps += 1;
        }
    }
    double total = 0.0;
    if (rc == LB_OK && hipStreamSynchronize(b->stream) != hipSuccess) rc = fail(LB_EHIP, "hipStreamSynchronize");
    for (int k = 0; k < n && rc == LB_OK; ++k) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]) != hipSuccess) rc = fail(LB_EHIP, "hipEventElapsedTime");
        total += t;
    }
    if (rc == LB_OK) *ms = total / n;
    return rc;
}

}  // extern "C"
