// Host runtime and C ABI of the D3Q19 lattice library (declared in include/lb.h).
//
// A lattice owns two population arrays (the pre- and post-collision arrays of
// the paper's fused scheme, Section 3.1), swapped by parity after every step,
// the neighbour masks used by bounce-back, and the buffers of the per-step
// FP64 conservation totals.  Work is enqueued on one in-order HIP stream;
// long step sequences are replayed from a captured HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lb.h"
#include "lb_host.h"
#include "lb_internal.h"

using namespace lbm;

// Scratch of lb_step_noalloc: the totals reduce's arrival ticket, the reduce
// workgroups' partials and the two buffers of step-workgroup partials, in one
// file-scope device array instead of the lattice's own allocations.  Every
// device holds its own copy at its own address; host code uses only that
// address (scratch_base), never the array's name.
constexpr size_t kScratchBytes = ((size_t)8 << 20) + ((size_t)64 << 10);  // 8 MiB + 64 KiB
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace lbm {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

long env_long(const char *name, long dflt)
{
    const char *v = getenv(name);
    if (!v || !*v) return dflt;
    return strtol(v, nullptr, 10);
}

}  // namespace lbm

namespace {

constexpr uint64_t kMagic = 0x4c42443351313921ull;  // "LBD3Q19!"
constexpr uint64_t kDead = 0xdeadd3a1deadd3a1ull;
// Requests of at least kGraphMin steps run as one captured graph of the whole
// run (up to kGraphMax steps per graph), kept for the next request of the
// same length.
constexpr int kGraphMin = 64;
constexpr int kGraphMax = 1024;


}  // namespace

struct lb_lattice {
    uint64_t magic;
    int nx, ny, nz;
    uint64_t n;       // sites
    Layout lay;       // storage layout of a population array
    uint64_t arr_elems;  // elements of one population array (19 * R * nx * blocks)
    int codec, esize;
    double tau, omega;
    double force[3];
    void *buf[2];
    void *alloc[2];   // allocations holding buf[0], buf[1] (buf[b] may sit at an offset)
    int cur;          // buf[cur] holds the state
    uint8_t *flags;   // device copy, or nullptr when all fluid
    float *ffield;    // per-site x-force added to force[0] (device, N floats), or nullptr
    uint32_t *nbmask;
    uint8_t *rowdirty;
    uint32_t *rowcum;
    bool solids;
    double n_fluid;
    double *partials;
    double *gpartials;
    unsigned int *ticket;
    double *ring;
    unsigned long long *counter;
    hipStream_t stream;
    int variant, vsites, grid, cus;
    int tile_order;
    int pull_nt;      // 1: plain steps with solids pull with non-temporal loads
    bool inplace;     // one population array (AA pattern); cur is then the phase (0 even, 1 odd)
    long long steps;
    RunGraphs graphs;
    std::vector<void *> adj_ws;  // state-sized buffers of the adjoint sweep, kept for later calls
    float *adj_mom;              // the sweep's per-step moments (adj_mom_steps x 4 N floats), kept likewise
    int adj_mom_steps;
    double *jval;     // device doubles: the outlet flux objective, then the parts of its sum
    int dev;          // HIP device the lattice lives on
    // scaled 16-bit storage (LB_S16): exponents, their device-side constants,
    // the two per-parity overflow flags and the last settled point (steps and
    // array) from which flagged steps are redone
    int s16e[3];      // exponents of the rest, axis and diagonal populations
    Scale16 sc;
    unsigned int *ovf;
    long long base_steps;
    int base_cur;
    long long rescales;
};

namespace {

int check(const lb_lattice *h)
{
    if (!h || h->magic != kMagic) return fail(LB_ESTATE, "invalid or destroyed lattice handle");
    return LB_OK;
}

// Arguments of a step (or adjoint step) of lattice h with the given kernel
// variant (its sites per lane set the tiling; -1: the lattice's own).
StepArgs step_args(const lb_lattice *h, int from, float *rho, float *u, int variant = -1)
{
    if (variant < 0) variant = h->variant;
    const int vsites = sites_per_thread(h->codec, variant);
    StepArgs a{};
    a.src = h->buf[from];
    a.dst = h->buf[from ^ 1];
    a.lay = h->lay;
    a.nx = h->nx;
    a.ny = h->ny;
    a.nz = h->nz;
    a.nslots = (int)(h->n / (uint64_t)vsites);
    // lanes per row (in-place lattices hold whole rows per tile); x-edge
    // elements pass through LDS within a tile (LB_LDS_EDGES=0: direct loads,
    // for comparison)
    const int row_lanes = h->nx / vsites;
    a.tile_order = h->tile_order;
    a.pull_nt = h->pull_nt;
    a.lds_edges = (variant != 0 && (h->inplace || env_long("LB_LDS_EDGES", 1) != 0)) ? 1 : 0;
    a.lg_row_lanes = 0;
    while ((1 << a.lg_row_lanes) < row_lanes) ++a.lg_row_lanes;
    a.div_pitch = make_fastdiv((uint32_t)h->nx);
    a.div_ny = make_fastdiv((uint32_t)h->ny);
    a.coll = make_coll((float)h->omega, (float)h->force[0], (float)h->force[1], (float)h->force[2]);
    a.nbmask = h->nbmask;
    a.rowdirty = h->rowdirty;
    a.rowcum = h->rowcum;
    a.rho_out = rho;
    a.u_out = u;
    a.partials = h->partials;
    a.fx_field = h->ffield;
    a.sc = h->sc;
    a.ovf = h->ovf;
    a.par = from;
    return a;
}

// Arguments of the macros kernel for the state in buf[cur] (in-place
// storage: the phase given by cur).
MacroArgs macro_args(const lb_lattice *h, int cur, float *rho, float *u)
{
    MacroArgs a{};
    a.src = h->buf[cur];
    a.lay = h->lay;
    a.n = (int)h->n;
    a.ny = h->ny;
    a.nz = h->nz;
    a.aa_phase = h->inplace ? (cur == 0 ? 1 : 2) : 0;
    a.fx = (float)h->force[0];
    a.fy = (float)h->force[1];
    a.fz = (float)h->force[2];
    a.flags = h->flags;
    a.fx_field = h->ffield;
    a.rho = rho;
    a.u = u;
    a.sc = h->sc;
    return a;
}

// Device buffers of the per-step totals: the step workgroups' partials (two
// buffers of grid slots, for runs of steps), the reduce workgroups' partials
// and the reduce's arrival ticket.
struct TotalsBufs {
    double *partials;
    double *gpartials;
    unsigned int *ticket;
};

TotalsBufs own_bufs(const lb_lattice *h) { return TotalsBufs{h->partials, h->gpartials, h->ticket}; }

// ---- the scratch array's address per device (resolved once per device, with
// that device current, when the first lattice is created on it)
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_base[kMaxDevices];

int resolve_scratch(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(LB_EHIP, "device %d beyond the library's %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_base[dev]) return LB_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
        return fail(LB_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_base[dev] = static_cast<unsigned char *>(p);
    return LB_OK;
}

unsigned char *scratch_base(int dev)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return (dev >= 0 && dev < kMaxDevices) ? g_scratch_base[dev] : nullptr;
}

// Scratch layout for lattice h: ticket (one 256-byte slot), the reduce
// workgroups' partials (4 doubles each, rounded up to 256 bytes), then two
// buffers of 4 doubles per step workgroup.
size_t scratch_gpart_bytes(const lb_lattice *h)
{
    const size_t ngroups = ((size_t)h->grid + kRedChunk - 1) / kRedChunk;
    return (ngroups * 4 * sizeof(double) + 255) & ~(size_t)255;
}

size_t scratch_need(const lb_lattice *h)
{
    return 256 + scratch_gpart_bytes(h) + (size_t)h->grid * 8 * sizeof(double);
}

TotalsBufs scratch_bufs(const lb_lattice *h, unsigned char *base)
{
    TotalsBufs tb;
    tb.ticket = reinterpret_cast<unsigned int *>(base);
    tb.gpartials = reinterpret_cast<double *>(base + 256);
    tb.partials = reinterpret_cast<double *>(base + 256 + scratch_gpart_bytes(h));
    return tb;
}

// Totals of the step whose workgroup partials are in buffer buf (0 or 1) and
// whose source array is buf[par] (its overflow flag, for scaled storage).
TotalsArgs totals_args(const lb_lattice *h, int buf, const TotalsBufs &tb, int par)
{
    TotalsArgs t{};
    t.ovf = h->codec == kS16 ? h->ovf + par : nullptr;
    t.partials = tb.partials + (size_t)buf * 4 * h->grid;
    t.nparts = h->grid;
    t.gpartials = tb.gpartials;
    t.ticket = tb.ticket;
    t.ring = h->ring;
    t.step_counter = h->counter;
    t.n_fluid = h->n_fluid;
    return t;
}

// ---- scaled 16-bit storage (LB_S16)

// Exponent of weight class c for the bound |g_i| <= w_i 2^m: the largest e
// with 32767 2^-e >= w_i 2^m, i.e. floor(log2(32767 / w_i)) - m (w = 1/3,
// 1/18, 1/36).
int s16_class_exponent(int c, int m) { return (c == 0 ? 16 : (c == 1 ? 19 : 20)) - m; }

void s16_set_class_exponents(lb_lattice *h, int m)
{
    for (int c = 0; c < 3; ++c) h->s16e[c] = s16_class_exponent(c, m);
}

void s16_update_scales(lb_lattice *h)
{
    for (int c = 0; c < 3; ++c) {
        const float d = std::ldexp(1.0f, -h->s16e[c]);
        h->sc.dm[c] = d;
        h->sc.da[c] = -8421376.0f * d;  // -(2^23 + 2^15) 2^-e: exact
        h->sc.em[c] = std::ldexp(1.0f, h->s16e[c]);
    }
    h->graphs.invalidate();  // the scales are launch arguments
}

constexpr int kS16MinExp = 4;   // widest range: |g| < 2^11
constexpr int kS16MaxExp = 60;  // narrowest range: |g| < 2^-45

int enqueue_steps(lb_lattice *h, int n, float *rho, float *u);

// count steps from buf[from] as one run with chained totals.  path (count + 1
// arrays, or NULL for the A/B pair): step k reads path[k] and writes
// path[k + 1].  mom (count pointers, or NULL): step k also writes its moments
// (one record rho, u_x, u_y, u_z per site, site order) to mom[k].
int enqueue_run(lb_lattice *h, int from, int count, hipStream_t s, const TotalsBufs &tb, void *const *path = nullptr,
                float *const *mom = nullptr);

// Wait for the lattice's work; if a scaled-storage step overflowed, widen
// the range of each weight class whose codes left it by one bit
// (re-encoding the intact source array of the first flagged step), and redo
// the flagged and skipped steps; repeat until no step is flagged.  Other
// codecs: no-op.
int settle(lb_lattice *h)
{
    if (h->codec != kS16) return LB_OK;
    for (;;) {
        unsigned int flag[2] = {0u, 0u};
        unsigned long long ctr = 0;
        HIP_OR_FAIL(hipMemcpyAsync(flag, h->ovf, sizeof flag, hipMemcpyDeviceToHost, h->stream));
        HIP_OR_FAIL(hipMemcpyAsync(&ctr, h->counter, sizeof ctr, hipMemcpyDeviceToHost, h->stream));
        HIP_OR_FAIL(hipStreamSynchronize(h->stream));
        if (!flag[0] && !flag[1]) {
            h->base_steps = h->steps;
            h->base_cur = h->cur;
            return LB_OK;
        }
        // the device counter counts the steps whose totals were appended:
        // exactly the steps before the first flagged one
        const long long good = (long long)ctr;
        const long long pending = h->steps - good;
        if (good < h->base_steps || pending < 1)
            return fail(LB_ESTATE, "scaled storage: inconsistent overflow record (%lld good of %lld steps)", good,
                        h->steps);
        // the overflowing step's class bits (the steps skipped after it add
        // only their skip bit)
        unsigned int classes = (flag[0] | flag[1]) & 7u;
        if (!classes) classes = 7u;
        Shift16 sh;
        for (int c = 0; c < 3; ++c) {
            sh.sh[c] = (classes >> c) & 1u;
            if (h->s16e[c] - sh.sh[c] < kS16MinExp)
                return fail(LB_EUNSTABLE, "scaled 16-bit storage: values beyond the widest range at step %lld "
                                          "(unstable run)", good + 1);
        }
        const int src = h->base_cur ^ (int)((good - h->base_steps) & 1);
        HIP_OR_FAIL(launch_s16_rescale(h->buf[src], h->lay, h->arr_elems, sh, h->stream));
        for (int c = 0; c < 3; ++c) h->s16e[c] -= sh.sh[c];
        s16_update_scales(h);
        HIP_OR_FAIL(launch_zero_words(h->ovf, 2, h->stream));
        h->cur = src;
        h->steps = good;
        h->base_steps = good;
        h->base_cur = src;
        h->rescales += 1;
        if (int rc = enqueue_steps(h, (int)pending, nullptr, nullptr)) return rc;
    }
}

// Enqueue one step from buf[from] on stream s.
int enqueue_one(lb_lattice *h, int from, float *rho, float *u, hipStream_t s, const TotalsBufs &tb)
{
    const bool macros = rho != nullptr;
    StepArgs a = step_args(h, from, rho, u);
    a.partials = tb.partials;
    if (h->inplace) {
        HIP_OR_FAIL(launch_aa_step(h->codec, h->variant, h->solids, from == 0, a, h->grid, s));
        HIP_OR_FAIL(launch_totals(totals_args(h, 0, tb, from), s));
        if (macros) HIP_OR_FAIL(launch_macros(h->codec, macro_args(h, from ^ 1, rho, u), s));
        return LB_OK;
    }
    HIP_OR_FAIL(launch_step(h->codec, h->variant, h->solids, macros, a, h->grid, s));
    HIP_OR_FAIL(launch_totals(totals_args(h, 0, tb, from), s));
    if (macros && h->solids && h->variant == 0)
        HIP_OR_FAIL(launch_zero_solid_macros(h->flags, (int)h->n, rho, u, s));
    return LB_OK;
}

// Enqueue count >= 1 steps without macros from buf[from] on stream s.  On
// the vector-row kernels the steps form a run: step k writes its workgroup
// partials into buffer k & 1, the first workgroup of step k + 1 appends the
// totals of step k, and one totals kernel closes the run.  The ring then
// holds the same values as with a totals kernel after every step.
int enqueue_run(lb_lattice *h, int from, int count, hipStream_t s, const TotalsBufs &tb, void *const *path,
                float *const *mom)
{
    if (h->inplace || h->variant == 0) {
        if (path || mom) return fail(LB_EINVAL, "explicit step buffers need the two-array row kernels");
        for (int k = 0; k < count; ++k) {
            int rc = enqueue_one(h, from ^ (k & 1), nullptr, nullptr, s, tb);
            if (rc) return rc;
        }
        return LB_OK;
    }
    for (int k = 0; k < count; ++k) {
        StepArgs a = step_args(h, from ^ (k & 1), mom ? mom[k] : nullptr, nullptr);
        a.mom_rec = mom ? 1 : 0;
        if (path) {
            a.src = path[k];
            a.dst = path[k + 1];
        }
        a.partials = tb.partials + (size_t)(k & 1) * 4 * h->grid;
        if (k > 0) a.prev = totals_args(h, (k - 1) & 1, tb, from ^ ((k - 1) & 1));
        HIP_OR_FAIL(launch_step(h->codec, h->variant, h->solids, mom != nullptr, a, h->grid, s));
    }
    HIP_OR_FAIL(launch_totals(totals_args(h, (count - 1) & 1, tb, from ^ ((count - 1) & 1)), s));
    return LB_OK;
}

// Capture the run of len steps from buf[parity] unless it is held already
// (a new length, or changed launch arguments, drops the held graphs).
int ensure_graph(lb_lattice *h, int len, int parity)
{
    RunGraphs &G = h->graphs;
    if (G.len != len) G.invalidate();
    if (!G.exec[parity]) {
        if (!G.cap) HIP_OR_FAIL(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
        HIP_OR_FAIL(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_run(h, parity, len, G.cap, own_bufs(h));
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
    }
    return LB_OK;
}

int run_graph(lb_lattice *h, int len, int parity)
{
    if (int rc = ensure_graph(h, len, parity)) return rc;
    HIP_OR_FAIL(hipGraphLaunch(h->graphs.exec[parity], h->stream));
    return LB_OK;
}

// Capture the graphs enqueue_steps(h, n) will replay, without launching them
// (keeps capture out of timed regions).
int prepare_graphs(lb_lattice *h, int n)
{
    if (n < kGraphMin) return LB_OK;
    const int len = std::min(n, kGraphMax);
    if (int rc = ensure_graph(h, len, h->cur)) return rc;
    if ((len & 1) && n >= 2 * len) return ensure_graph(h, len, h->cur ^ 1);
    return LB_OK;
}

int enqueue_steps(lb_lattice *h, int n, float *rho, float *u)
{
    int plain = rho ? n - 1 : n;
    if (plain >= kGraphMin) {
        const int len = std::min(plain, kGraphMax);
        while (plain >= len) {
            if (int rc = run_graph(h, len, h->cur)) return rc;
            h->cur ^= len & 1;
            h->steps += len;
            plain -= len;
        }
    }
    if (plain > 0) {
        int rc = enqueue_run(h, h->cur, plain, h->stream, own_bufs(h));
        if (rc) return rc;
        h->cur ^= plain & 1;
        h->steps += plain;
    }
    if (rho) {
        int rc = enqueue_one(h, h->cur, rho, u, h->stream, own_bufs(h));
        if (rc) return rc;
        h->cur ^= 1;
        h->steps += 1;
    }
    return LB_OK;
}

void release(lb_lattice *h)
{
    h->graphs.release();
    void *ptrs[] = {h->alloc[0], h->alloc[1], h->flags,   h->nbmask, h->rowdirty, h->rowcum,
                    h->partials, h->gpartials, h->ticket, h->ring,  h->counter, h->ffield, h->jval,
                    h->ovf};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (void *p : h->adj_ws) (void)hipFree(p);
    h->adj_ws.clear();
    if (h->adj_mom) (void)hipFree(h->adj_mom);
    h->adj_mom = nullptr;
    h->adj_mom_steps = 0;
}

int create_impl(lb_lattice **out, int nx, int ny, int nz, double tau, const uint8_t *flags, int storage,
                void *stream)
{
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return fail(LB_EINVAL, "lattice extents must be >= 1 (got %d x %d x %d)", nx, ny, nz);
    const uint64_t n = (uint64_t)nx * ny * nz;
    if (n > 0x7fffffffull - 4096) return fail(LB_EINVAL, "lattice of %llu sites exceeds 2^31 - 4097", (unsigned long long)n);
    if (!(tau > 0.5)) return fail(LB_EINVAL, "tau must be > 0.5 or +inf (got %g)", tau);
    const bool inplace = (storage & LB_INPLACE) != 0;
    storage &= ~LB_INPLACE;
    if (storage != LB_F32 && storage != LB_F16S && storage != LB_BF16S && storage != LB_S16)
        return fail(LB_EINVAL, "unknown storage codec %d", storage);
    if (inplace && storage == LB_S16) return fail(LB_EINVAL, "scaled 16-bit storage needs two arrays (no LB_INPLACE)");
    uint64_t nsolid = 0;
    if (flags) {
        for (uint64_t s = 0; s < n; ++s) {
            if (flags[s] > 1) return fail(LB_EINVAL, "flag value %d at site %llu (allowed: 0 fluid, 1 solid)", (int)flags[s], (unsigned long long)s);
            nsolid += flags[s];
        }
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(LB_EHIP, "no HIP device available");

    lb_lattice *h = new (std::nothrow) lb_lattice();
    if (!h) return fail(LB_ENOMEM, "host allocation failed");
    h->nx = nx;
    h->ny = ny;
    h->nz = nz;
    h->n = n;
    h->codec = storage;
    h->esize = storage == LB_F32 ? 4 : 2;
    h->tau = tau;
    h->omega = std::isinf(tau) ? 0.0 : 1.0 / tau;
    h->stream = reinterpret_cast<hipStream_t>(stream);
    h->solids = nsolid > 0;
    h->n_fluid = (double)(n - nsolid);
    h->inplace = inplace;

    // Step kernel: vector rows with 16-byte accesses (FP32: 4 sites per lane,
    // FP16/BF16: 8) or, for the scaled 16-bit codec, 8-byte accesses (4
    // sites: its 16-byte kernel runs at two waves per SIMD); narrower vectors
    // when nx is not a multiple of the width, one site per thread when no
    // vector width divides nx.  LB_KERNEL (0..3) overrides the choice.
    const long kernel = env_long("LB_KERNEL", -1);
    int variant = storage == LB_S16 ? 2 : 1;
    if (kernel >= 0 && kernel <= 3) variant = (int)kernel;
    else if (kernel != -1) {
        delete h;
        return fail(LB_EINVAL, "LB_KERNEL must be 0, 1, 2 or 3");
    }
    if (variant != 0 && nx % sites_per_thread(storage, variant) != 0) {
        if (kernel > 0) {
            delete h;
            return fail(LB_EINVAL, "kernel %d needs nx %% %d == 0", variant, sites_per_thread(storage, variant));
        }
        int v = variant + 1;
        while (v <= 3 && nx % sites_per_thread(storage, v) != 0) ++v;
        variant = v <= 3 ? v : 0;
    }
    if (inplace) {
        // the in-place push exchanges x-edges inside a tile: whole rows per
        // tile, i.e. nx / V a power of two of at most 256 lanes
        auto rows_fit = [&](int v) {
            if (v < 1 || v > 3) return false;
            const int V = sites_per_thread(storage, v);
            return nx % V == 0 && nx / V <= kBlock && kBlock % (nx / V) == 0;
        };
        int v = variant == 0 ? 1 : variant;
        while (v <= 3 && !rows_fit(v)) ++v;
        if (v > 3) {
            delete h;
            return fail(LB_EINVAL, "in-place storage needs nx = V * 2^k with nx / V <= 256 (V = sites per lane); got nx = %d", nx);
        }
        variant = v;
    }
    h->variant = variant;
    h->vsites = sites_per_thread(storage, h->variant);
    // Storage blocks of R rows: by default the largest power of two with
    // R * nx * bytes <= 32 KiB per population segment.  LB_BLOCK_ROWS (a power
    // of two) overrides it for tuning.
    const uint64_t nrows = (uint64_t)ny * nz;
    long rows = env_long("LB_BLOCK_ROWS", 0);
    if (rows < 0 || (rows & (rows - 1)) != 0) {
        delete h;
        return fail(LB_EINVAL, "LB_BLOCK_ROWS must be a power of two");
    }
    if (rows == 0) {
        rows = 1;
        while ((uint64_t)(rows * 2) * nx * h->esize <= 32768 && (uint64_t)rows < nrows) rows *= 2;
    }
    uint32_t lg = 0;
    while ((1l << lg) < rows) ++lg;
    h->lay.nx = (uint32_t)nx;
    h->lay.pitch = (uint32_t)nx;
    h->lay.lg_r = lg;
    // LB_SEG_PAD elements (a multiple of 128, so every vector stays aligned)
    // between the population segments of a block, for tuning
    const long seg_pad = env_long("LB_SEG_PAD", 0);
    if (seg_pad < 0 || seg_pad % 128 != 0) {
        delete h;
        return fail(LB_EINVAL, "LB_SEG_PAD must be a non-negative multiple of 128");
    }
    const uint64_t seg = (uint64_t)rows * nx + (uint64_t)seg_pad;
    if (!block_fits(seg, kQ, h->esize)) {
        delete h;
        return fail(LB_EINVAL, "a storage block of %llu elements per population (rows of %d sites) reaches 1 GiB",
                    (unsigned long long)seg, nx);
    }
    h->lay.seg = (uint32_t)seg;
    h->lay.blk = (uint32_t)(kQ * seg);
    const uint64_t nblocks = (nrows + rows - 1) / rows;
    h->arr_elems = nblocks * h->lay.blk;

    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete h;
        return fail(LB_EHIP, "cannot query the HIP device");
    }
    h->cus = prop.multiProcessorCount;
    h->dev = dev;
    if (int rc = resolve_scratch(dev)) {
        delete h;
        return rc;
    }
    // One workgroup per tile of kBlock lanes (the vector-row step kernels
    // take exactly one tile each: nothing is carried from tile to tile, which
    // keeps their register budget to one tile's values).  n <= 2^31 sites, so
    // the tile count fits the grid.
    const uint64_t tiles = (n / h->vsites + kBlock - 1) / kBlock;
    h->grid = (int)(tiles < 1 ? 1 : tiles);

    auto bail = [&](int code, const char *what, hipError_t e) {
        release(h);
        delete h;
        return fail(code, "%s: %s", what, hipGetErrorString(e));
    };
    const size_t pbytes = (size_t)h->arr_elems * h->esize;
    // LB_AB_OFFSET bytes (a multiple of 256) in front of the second array, for
    // tuning the relative placement of the two arrays in the HBM channels
    const long ab_off = env_long("LB_AB_OFFSET", 0);
    if (ab_off < 0 || ab_off % 256 != 0) return bail(LB_EINVAL, "LB_AB_OFFSET", hipErrorInvalidValue);
    {
        const long o = env_long("LB_TILE_ORDER", 0);
        h->tile_order = o >= 0 && o <= 2 ? (int)o : 0;
    }
    h->pull_nt = env_long("LB_PULL_NT", 0) != 0 ? 1 : 0;
    hipError_t e;
    for (int b = 0; b < (h->inplace ? 1 : 2); ++b) {
        const size_t off = b == 1 ? (size_t)ab_off : 0;
        e = hipMalloc(&h->alloc[b], pbytes + off);
        if (e != hipSuccess) return bail(LB_ENOMEM, "hipMalloc(populations)", e);
        h->buf[b] = static_cast<char *>(h->alloc[b]) + off;
        e = hipMemsetAsync(h->buf[b], 0, pbytes, h->stream);
        if (e != hipSuccess) return bail(LB_EHIP, "hipMemsetAsync", e);
    }
    if (h->inplace) h->buf[1] = h->buf[0];  // steps read and write the one array
    // per-step totals: one slot per step workgroup (two buffers, for runs of
    // steps) and one per reduce workgroup
    const size_t ngroups = ((size_t)h->grid + kRedChunk - 1) / kRedChunk;
    if ((e = hipMalloc(&h->partials, (size_t)h->grid * 8 * sizeof(double))) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc", e);
    if ((e = hipMalloc(&h->gpartials, ngroups * 4 * sizeof(double))) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc", e);
    if ((e = hipMalloc(&h->ticket, sizeof(unsigned int))) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc", e);
    if ((e = hipMalloc(&h->ring, (size_t)kRingCap * 4 * sizeof(double))) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc", e);
    if ((e = hipMalloc(&h->counter, sizeof(unsigned long long))) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc", e);
    // J, then the per-workgroup parts of its sum
    if ((e = hipMalloc(&h->jval, (1 + (size_t)outlet_parts(ny, nz)) * sizeof(double))) != hipSuccess)
        return bail(LB_ENOMEM, "hipMalloc", e);
    if ((e = hipMemsetAsync(h->ticket, 0, sizeof(unsigned int), h->stream)) != hipSuccess) return bail(LB_EHIP, "hipMemsetAsync", e);
    if ((e = hipMemsetAsync(h->counter, 0, sizeof(unsigned long long), h->stream)) != hipSuccess) return bail(LB_EHIP, "hipMemsetAsync", e);
    if ((e = hipMemsetAsync(h->ring, 0, (size_t)kRingCap * 4 * sizeof(double), h->stream)) != hipSuccess) return bail(LB_EHIP, "hipMemsetAsync", e);
    if (storage == LB_S16) {
        // two per-parity overflow flags and three words for the initial maxima
        if ((e = hipMalloc(&h->ovf, 8 * sizeof(unsigned int))) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc", e);
        if ((e = hipMemsetAsync(h->ovf, 0, 8 * sizeof(unsigned int), h->stream)) != hipSuccess) return bail(LB_EHIP, "hipMemsetAsync", e);
        s16_set_class_exponents(h, -4);  // |g_i| <= w_i / 16 until lb_init_eq sizes the ranges
        s16_update_scales(h);
    }
    if (h->solids) {
        if ((e = hipMalloc(&h->flags, n)) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc(flags)", e);
        if ((e = hipMalloc(&h->nbmask, n * sizeof(uint32_t) + 64)) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc(masks)", e);
        if ((e = hipMalloc(&h->rowdirty, (size_t)ny * nz)) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc(rows)", e);
        if ((e = hipMalloc(&h->rowcum, ((size_t)ny * nz + 1) * sizeof(uint32_t))) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc(rows)", e);
        if ((e = hipMemcpyAsync(h->flags, flags, n, hipMemcpyHostToDevice, h->stream)) != hipSuccess) return bail(LB_EHIP, "hipMemcpyAsync(flags)", e);
        if ((e = launch_masks(h->flags, nx, ny, nz, nx, h->nbmask, h->rowdirty, h->rowcum, h->stream)) != hipSuccess) return bail(LB_EHIP, "mask kernels", e);
    }
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return bail(LB_EHIP, "hipStreamSynchronize", e);
    h->magic = kMagic;
    *out = h;
    return LB_OK;
}

}  // namespace

extern "C" {

const char *lb_last_error(void) { return g_err.c_str(); }

lb_lattice *lb_create_ex(int nx, int ny, int nz, double tau, const uint8_t *flags, int storage, void *hip_stream)
{
    lb_lattice *h = nullptr;
    try {
        if (create_impl(&h, nx, ny, nz, tau, flags, storage, hip_stream) != LB_OK) return nullptr;
    } catch (...) {
        fail(LB_ENOMEM, "unexpected exception in lb_create");
        return nullptr;
    }
    g_err.clear();
    return h;
}

lb_lattice *lb_create(int nx, int ny, int nz, double tau, const uint8_t *flags)
{
    return lb_create_ex(nx, ny, nz, tau, flags, LB_F32, nullptr);
}

void lb_destroy(lb_lattice *h)
{
    if (!h || h->magic != kMagic) return;
    (void)hipStreamSynchronize(h->stream);
    h->magic = kDead;
    release(h);
    delete h;
}

int lb_set_force(lb_lattice *h, double fx, double fy, double fz)
{
    if (int rc = check(h)) return rc;
    if (!std::isfinite(fx) || !std::isfinite(fy) || !std::isfinite(fz)) return fail(LB_EINVAL, "force must be finite");
    h->force[0] = fx;
    h->force[1] = fy;
    h->force[2] = fz;
    h->graphs.invalidate();
    return LB_OK;
}

int lb_init_eq(lb_lattice *h, const double *rho, const double *u)
{
    if (int rc = check(h)) return rc;
    InitArgs a{};
    a.dst = h->buf[0];
    a.lay = h->lay;
    a.n = (int)h->n;
    a.rho = rho;
    a.u = u;
    a.flags = h->flags;
    a.swap = h->inplace ? 1 : 0;
    if (h->codec == kS16) {
        // size the ranges from the initial state: |g_i| <= w_i 2^m with
        // 2^m >= 2 max |g_i^eq| / w_i (one bit of headroom); later growth is
        // caught by the overflow flags
        HIP_OR_FAIL(launch_eq_absmax(a, h->ovf + 2, h->stream));
        unsigned int bits[3] = {0u, 0u, 0u};
        HIP_OR_FAIL(hipMemcpyAsync(bits, h->ovf + 2, sizeof bits, hipMemcpyDeviceToHost, h->stream));
        HIP_OR_FAIL(hipStreamSynchronize(h->stream));
        for (int c = 0; c < 3; ++c) {
            float mx = 0.0f;
            std::memcpy(&mx, &bits[c], sizeof mx);
            if (!std::isfinite(mx)) return fail(LB_EINVAL, "initial fields are not finite");
            // one bit of headroom; at rest (mx = 0) the class gets |g| <= w / 16.
            // (Four bits for the rest population would avoid the widenings of
            // the first steps from a noisy velocity field, but its coarser step
            // then costs more accuracy than the widenings cost time.)
            int m = mx > 0.0f ? (int)std::ceil(std::log2(2.0 * (double)mx)) : -4;
            m = std::min(3, std::max(-30, m));
            h->s16e[c] = s16_class_exponent(c, m);
        }
        s16_update_scales(h);
        a.sc = h->sc;
        HIP_OR_FAIL(launch_zero_words(h->ovf, 2, h->stream));
    }
    HIP_OR_FAIL(launch_init(h->codec, a, h->stream));
    HIP_OR_FAIL(hipMemsetAsync(h->counter, 0, sizeof(unsigned long long), h->stream));
    h->cur = 0;
    h->steps = 0;
    h->base_steps = 0;
    h->base_cur = 0;
    return LB_OK;
}

int lb_step(lb_lattice *h, int n)
{
    if (int rc = check(h)) return rc;
    if (n < 0) return fail(LB_EINVAL, "step count must be >= 0 (got %d)", n);
    return enqueue_steps(h, n, nullptr, nullptr);
}

int lb_step_noalloc(lb_lattice *h, int n)
{
    if (int rc = check(h)) return rc;
    if (n < 0) return fail(LB_EINVAL, "step count must be >= 0 (got %d)", n);
    const size_t need = scratch_need(h);
    if (need > kScratchBytes)
        return fail(LB_EINVAL,
                    "lb_step_noalloc: the totals of this lattice need %zu bytes of scratch (%d step workgroups); "
                    "the library's static scratch holds %zu bytes",
                    need, h->grid, kScratchBytes);
    if (n == 0) return LB_OK;
    unsigned char *base = scratch_base(h->dev);
    if (!base) return fail(LB_ESTATE, "scratch address of device %d not resolved", h->dev);
    const TotalsBufs tb = scratch_bufs(h, base);
    // the ticket must start at zero: a kernel, not a memset, clears it
    HIP_OR_FAIL(launch_zero_words(tb.ticket, 1, h->stream));
    if (int rc = enqueue_run(h, h->cur, n, h->stream, tb)) return rc;
    h->cur ^= n & 1;
    h->steps += n;
    return LB_OK;
}

int lb_step_macros(lb_lattice *h, int n, float *rho, float *u)
{
    if (int rc = check(h)) return rc;
    if (n < 1) return fail(LB_EINVAL, "lb_step_macros needs n >= 1 (got %d)", n);
    if (!rho || !u) return fail(LB_EINVAL, "rho and u must be device pointers");
    if (h->codec == kS16) {
        // the fields of the settled state (a redone step must not leave its
        // first attempt's fields behind)
        if (int rc = enqueue_steps(h, n, nullptr, nullptr)) return rc;
        if (int rc = settle(h)) return rc;
        HIP_OR_FAIL(launch_macros(h->codec, macro_args(h, h->cur, rho, u), h->stream));
        return LB_OK;
    }
    return enqueue_steps(h, n, rho, u);
}

int lb_macros(lb_lattice *h, float *rho, float *u)
{
    if (int rc = check(h)) return rc;
    if (int rc = settle(h)) return rc;
    HIP_OR_FAIL(launch_macros(h->codec, macro_args(h, h->cur, rho, u), h->stream));
    return LB_OK;
}

int lb_set_force_field(lb_lattice *h, const float *fx)
{
    if (int rc = check(h)) return rc;
    if (!fx) {
        HIP_OR_FAIL(hipStreamSynchronize(h->stream));
        if (h->ffield) (void)hipFree(h->ffield);
        h->ffield = nullptr;
        h->graphs.invalidate();
        return LB_OK;
    }
    if (h->codec != kF32) return fail(LB_EINVAL, "force fields need FP32 storage");
    if (h->inplace) return fail(LB_EINVAL, "force fields need two-array storage");
    if (!h->ffield) {
        hipError_t e = hipMalloc(&h->ffield, h->n * sizeof(float) + 64);
        if (e != hipSuccess) {
            h->ffield = nullptr;
            return fail(LB_ENOMEM, "hipMalloc(force field): %s", hipGetErrorString(e));
        }
    }
    HIP_OR_FAIL(hipMemcpyAsync(h->ffield, fx, h->n * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    // the field is read as whole vectors of the row kernels: any nx works with one site per lane
    if (h->variant == 0) {
        h->variant = 3;
        h->vsites = sites_per_thread(h->codec, 3);
        const uint64_t tiles = (h->n / h->vsites + kBlock - 1) / kBlock;
        h->grid = (int)std::min<uint64_t>(tiles, 0x7fffffffull);
        HIP_OR_FAIL(hipStreamSynchronize(h->stream));
        (void)hipFree(h->partials);
        (void)hipFree(h->gpartials);
        h->partials = h->gpartials = nullptr;
        const size_t ngroups = ((size_t)h->grid + kRedChunk - 1) / kRedChunk;
        if (hipMalloc(&h->partials, (size_t)h->grid * 8 * sizeof(double)) != hipSuccess ||
            hipMalloc(&h->gpartials, ngroups * 4 * sizeof(double)) != hipSuccess)
            return fail(LB_ENOMEM, "hipMalloc(partials)");
    }
    h->graphs.invalidate();
    return LB_OK;
}

}  // extern "C"

namespace {

OutletArgs outlet_args(const lb_lattice *h, const void *state)
{
    OutletArgs a{};
    a.state = state;
    a.J = h->jval;
    a.part = h->jval + 1;
    a.lay = h->lay;
    a.nx = h->nx;
    a.ny = h->ny;
    a.nz = h->nz;
    a.flags = h->flags;
    a.fx = (float)h->force[0];
    a.fx_field = h->ffield;
    return a;
}

// The outlet flux of the state in buf[h->cur] into *J (host); synchronises.
int outlet_flux_value(lb_lattice *h, double *J)
{
    HIP_OR_FAIL(launch_outlet_flux(h->codec, outlet_args(h, h->buf[h->cur]), h->stream));
    HIP_OR_FAIL(hipMemcpyAsync(J, h->jval, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_OR_FAIL(hipStreamSynchronize(h->stream));
    return LB_OK;
}

// Checkpointed adjoint sweep of nsteps steps.  The objective's seed dJ/dS_N
// is the caller's raw planes (seed != nullptr) or the outlet flux's (seed ==
// nullptr, which also adds the flux's direct term and stores J in *J when J
// is not null).
int grad_impl(lb_lattice *h, int nsteps, int every, const float *seed, float *grad, double *J)
{
    if (int rc = check(h)) return rc;
    if (h->codec != kF32) return fail(LB_EINVAL, "the adjoint needs FP32 storage");
    if (h->inplace) return fail(LB_EINVAL, "the adjoint needs two-array storage");
    if (nsteps < 1 || every < 1) return fail(LB_EINVAL, "nsteps and every must be >= 1");
    if (!grad) return fail(LB_EINVAL, "grad must be a device pointer");
    if (h->variant == 0) return fail(LB_EINVAL, "the adjoint runs the row kernels: set a force field first");
    // sites per lane of the adjoint kernel: one (4-byte accesses) ran fastest
    // on the porous channels; LB_ADJ_KERNEL (1, 2, 3: four, two, one) overrides
    int av = (int)env_long("LB_ADJ_KERNEL", 0);
    if (av < 1 || av > 3) av = 3;
    while (av < 3 && h->nx % sites_per_thread(kF32, av) != 0) ++av;
    const int adj_grid = (int)std::min<uint64_t>((h->n / sites_per_thread(kF32, av) + kBlock - 1) / kBlock, 0x7fffffffull);
    const size_t abytes = (size_t)h->arr_elems * sizeof(float);
    const int nck = (nsteps + every - 1) / every;
    const int seg = std::min(every, nsteps);
    // Device memory of the sweep: the checkpoints, two states for the
    // recomputed stretches, the two adjoint arrays (the first also takes the
    // seed), and the moments of one stretch's steps (a 16-byte record per
    // site and step).  The buffers are kept by the lattice and reused by
    // later calls that need no more of them.
    const size_t need = (size_t)nck + 4;
    while (h->adj_ws.size() < need) {
        void *p = nullptr;
        if (hipMalloc(&p, abytes) != hipSuccess)
            return fail(LB_ENOMEM, "hipMalloc of the adjoint sweep (%zu states of %zu bytes)", need, abytes);
        h->adj_ws.push_back(p);
    }
    if (h->adj_mom_steps < seg) {
        HIP_OR_FAIL(hipStreamSynchronize(h->stream));
        if (h->adj_mom) (void)hipFree(h->adj_mom);
        h->adj_mom = nullptr;
        h->adj_mom_steps = 0;
        void *p = nullptr;
        if (hipMalloc(&p, (size_t)seg * 4 * h->n * sizeof(float)) != hipSuccess)
            return fail(LB_ENOMEM, "hipMalloc of the adjoint sweep's moments (%d steps of %zu sites)", seg,
                        (size_t)h->n);
        h->adj_mom = static_cast<float *>(p);
        h->adj_mom_steps = seg;
    }
    size_t next = 0;
    auto grab = [&]() { return static_cast<char *>(h->adj_ws[next++]); };
    std::vector<char *> ck(nck);
    for (int k = 0; k < nck; ++k) ck[k] = grab();
    char *tmp[2] = {grab(), grab()};
    char *nu[2] = {grab(), grab()};
    std::vector<float *> mom(seg);
    for (int j = 0; j < seg; ++j) mom[j] = h->adj_mom + (size_t)j * 4 * h->n;
    int rc = LB_OK;
    auto hip = [&](hipError_t e, const char *what) {
        if (rc == LB_OK && e != hipSuccess) rc = fail(LB_EHIP, "%s: %s", what, hipGetErrorString(e));
    };
    // Forward: the ordinary steps as runs with chained totals, one run per
    // stretch.  Each stretch starts from its checkpoint and its last step
    // writes the next checkpoint (the first is a copy of the starting
    // state), so no checkpoint is copied; the last stretch ends in the
    // lattice's array for step nsteps and also writes the moments of its
    // steps, so the backward pass need not recompute it.
    const int final_cur = h->cur ^ (nsteps & 1);
    hip(hipMemcpyAsync(ck[0], h->buf[h->cur], abytes, hipMemcpyDeviceToDevice, h->stream), "checkpoint");
    for (int k = 0; k < nck && rc == LB_OK; ++k) {
        const int len = std::min(every, nsteps - k * every);
        const bool last = k == nck - 1;
        std::vector<void *> path(len + 1);
        path[0] = ck[k];
        for (int j = 1; j < len; ++j) path[j] = tmp[j & 1];
        path[len] = last ? h->buf[final_cur] : ck[k + 1];
        rc = enqueue_run(h, h->cur, len, h->stream, own_bufs(h), path.data(), last ? mom.data() : nullptr);
    }
    if (rc == LB_OK) {
        h->cur = final_cur;
        h->steps += nsteps;
    }
    // the objective of the final state: J, and its seed dJ/dS_N (storage
    // layout) in the first adjoint array
    if (rc == LB_OK && !seed && J) rc = outlet_flux_value(h, J);
    if (rc == LB_OK) hip(hipMemsetAsync(nu[0], 0, abytes, h->stream), "hipMemsetAsync");
    if (rc == LB_OK) {
        if (seed) {
            hip(launch_repack(const_cast<float *>(seed), nu[0], h->lay, (int64_t)h->n, 4, true, h->stream), "seed");
        } else {
            OutletArgs oa = outlet_args(h, nullptr);
            oa.seed = reinterpret_cast<float *>(nu[0]);
            hip(launch_outlet_seed(oa, h->stream), "outlet seed");
        }
    }
    if (rc == LB_OK) hip(hipMemsetAsync(grad, 0, h->n * sizeof(float), h->stream), "hipMemsetAsync");
    if (rc == LB_OK) hip(hipMemsetAsync(nu[1], 0, abytes, h->stream), "hipMemsetAsync");
    // Backward, stretch by stretch from the last.  Each stretch but the last
    // is recomputed from its checkpoint through the two scratch states,
    // keeping only its steps' moments (recomputed steps write no totals);
    // the adjoint steps then run backwards through those moments.
    int cur_nu = 0;
    bool first = true;
    for (int k = nck - 1; k >= 0 && rc == LB_OK; --k) {
        const int start = k * every, stop = std::min(start + every, nsteps);
        for (int j = 0; j < stop - start && rc == LB_OK && k < nck - 1; ++j) {
            StepArgs a = step_args(h, 0, mom[j], nullptr);
            a.mom_rec = 1;
            a.src = j == 0 ? ck[k] : tmp[(j - 1) & 1];
            // the stretch's last state is not needed: that step writes its moments only
            a.dst = j + 1 < stop - start ? tmp[j & 1] : nullptr;
            hip(launch_step(h->codec, h->variant, h->solids, true, a, h->grid, h->stream), "recompute step");
        }
        for (int n = stop - 1; n >= start && rc == LB_OK; --n) {
            AdjArgs a{};
            a.s = step_args(h, 0, nullptr, nullptr, av);
            a.mom = mom[n - start];
            a.lam_in = nu[cur_nu];
            a.nu_out = nu[cur_nu ^ 1];
            a.grad = grad;
            hip(launch_adjoint(av, first, a, adj_grid, h->stream), "adjoint step");
            first = false;
            cur_nu ^= 1;
        }
    }
    if (rc == LB_OK && !seed) {
        OutletArgs oa = outlet_args(h, nullptr);
        oa.grad = grad;
        hip(launch_outlet_direct(oa, h->stream), "outlet direct term");
    }
    (void)hipStreamSynchronize(h->stream);
    return rc;
}

}  // namespace

extern "C" {

int lb_grad_force_x(lb_lattice *h, int nsteps, int every, const float *seed, float *grad)
{
    if (int rc = check(h)) return rc;
    if (!seed) return fail(LB_EINVAL, "seed must be a device pointer");
    return grad_impl(h, nsteps, every, seed, grad, nullptr);
}

int lb_grad_outlet_flux_x(lb_lattice *h, int nsteps, int every, float *grad, double *J)
{
    if (int rc = check(h)) return rc;
    return grad_impl(h, nsteps, every, nullptr, grad, J);
}

int lb_outlet_flux(lb_lattice *h, double *J)
{
    if (int rc = check(h)) return rc;
    if (!J) return fail(LB_EINVAL, "J must be a host pointer");
    if (h->inplace) return fail(LB_EINVAL, "the outlet flux needs two-array storage");
    if (h->codec == kS16) return fail(LB_EINVAL, "the outlet flux needs FP32, FP16 or BF16 storage");
    return outlet_flux_value(h, J);
}


int lb_sums(lb_lattice *h, double *out, int k)
{
    if (int rc = check(h)) return rc;
    if (k < 0 || !out) return fail(LB_EINVAL, "bad output buffer or k");
    const long long avail = h->steps < kRingCap ? h->steps : kRingCap;
    if (k > avail) return fail(LB_EINVAL, "asked for %d step totals, %lld available", k, avail);
    if (int rc = settle(h)) return rc;
    HIP_OR_FAIL(hipStreamSynchronize(h->stream));
    std::vector<double> ring((size_t)kRingCap * 4);
    HIP_OR_FAIL(hipMemcpy(ring.data(), h->ring, ring.size() * sizeof(double), hipMemcpyDeviceToHost));
    bool bad = false;
    for (int j = 0; j < k; ++j) {
        const long long step = h->steps - k + j;
        const double *r = &ring[4 * (size_t)(step % kRingCap)];
        for (int c = 0; c < 4; ++c) {
            out[4 * j + c] = r[c];
            if (!std::isfinite(r[c])) bad = true;
        }
    }
    if (bad) return fail(LB_EUNSTABLE, "conservation totals contain NaN or Inf");
    return LB_OK;
}

static int copy_f(lb_lattice *h, void *host_or_dev, size_t bytes, int where, bool to_lattice)
{
    if (int rc = check(h)) return rc;
    if (int rc = settle(h)) return rc;
    const size_t want = (size_t)kQ * h->n * h->esize;
    if (bytes != want) return fail(LB_EINVAL, "buffer is %zu bytes, expected %zu", bytes, want);
    if (!host_or_dev) return fail(LB_EINVAL, "NULL buffer");
    if (where != LB_HOST && where != LB_DEVICE) return fail(LB_EINVAL, "where must be LB_HOST or LB_DEVICE");
    if (h->inplace) {
        // in-place storage: the state is rebuilt from (or written into) the
        // array by a kernel; writing leaves the array in the even form
        void *planes = host_or_dev;
        hipError_t e = hipSuccess;
        if (where == LB_HOST) {
            e = hipMalloc(&planes, bytes);
            if (e != hipSuccess) return fail(LB_ENOMEM, "hipMalloc(staging): %s", hipGetErrorString(e));
            if (to_lattice) e = hipMemcpyAsync(planes, host_or_dev, bytes, hipMemcpyHostToDevice, h->stream);
        }
        if (e == hipSuccess)
            e = launch_aa_planes(planes, h->buf[0], h->lay, h->ny, h->nz, h->flags, h->esize, h->cur == 0 ? 1 : 2,
                                 to_lattice, h->stream);
        if (e == hipSuccess && where == LB_HOST && !to_lattice)
            e = hipMemcpyAsync(host_or_dev, planes, bytes, hipMemcpyDeviceToHost, h->stream);
        if (where == LB_HOST) {
            const hipError_t se = hipStreamSynchronize(h->stream);
            (void)hipFree(planes);
            if (e == hipSuccess) e = se;
        }
        if (e != hipSuccess) return fail(LB_EHIP, "population copy: %s", hipGetErrorString(e));
        if (to_lattice) {
            h->cur = 0;
            h->graphs.invalidate();
        }
        return LB_OK;
    }
    // population i: full blocks as one 2-D copy (R rows per block), then the
    // rows of a last, partly filled block
    const size_t es = (size_t)h->esize;
    const uint64_t rows = 1ull << h->lay.lg_r;
    const size_t seg = h->lay.seg * es, blk = h->lay.blk * es, plane = h->n * es;
    const size_t width = (size_t)rows * h->nx * es;  // bytes of one population in a full block
    const uint64_t nrows = (uint64_t)h->ny * h->nz;
    const uint64_t nfull = nrows / rows;
    const size_t tail = (size_t)(nrows - nfull * rows) * h->nx * es;
    char *state = reinterpret_cast<char *>(h->buf[h->cur]);
    char *user = reinterpret_cast<char *>(host_or_dev);
    hipMemcpyKind kind = where == LB_HOST ? (to_lattice ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost)
                                          : hipMemcpyDeviceToDevice;
    for (int i = 0; i < kQ; ++i) {
        char *lat = state + (size_t)i * seg;
        char *usr = user + (size_t)i * plane;
        if (nfull > 0) {
            if (to_lattice)
                HIP_OR_FAIL(hipMemcpy2DAsync(lat, blk, usr, width, width, nfull, kind, h->stream));
            else
                HIP_OR_FAIL(hipMemcpy2DAsync(usr, width, lat, blk, width, nfull, kind, h->stream));
        }
        if (tail > 0) {
            char *lt = lat + nfull * blk;
            char *ut = usr + nfull * width;
            HIP_OR_FAIL(hipMemcpyAsync(to_lattice ? lt : ut, to_lattice ? ut : lt, tail, kind, h->stream));
        }
    }
    if (where == LB_HOST) HIP_OR_FAIL(hipStreamSynchronize(h->stream));
    return LB_OK;
}

int lb_get_f(lb_lattice *h, void *buf, size_t bytes, int where) { return copy_f(h, buf, bytes, where, false); }

int lb_set_f(lb_lattice *h, const void *buf, size_t bytes, int where)
{
    const int rc = copy_f(h, const_cast<void *>(buf), bytes, where, true);
    if (rc == LB_OK) {
        h->base_steps = h->steps;
        h->base_cur = h->cur;
    }
    return rc;
}

int lb_sync(lb_lattice *h)
{
    if (int rc = check(h)) return rc;
    if (int rc = settle(h)) return rc;
    HIP_OR_FAIL(hipStreamSynchronize(h->stream));
    return LB_OK;
}

int lb_get_scales(lb_lattice *h, int *exps)
{
    if (int rc = check(h)) return rc;
    if (h->codec != kS16) return fail(LB_EINVAL, "scales exist for LB_S16 storage only");
    if (!exps) return fail(LB_EINVAL, "NULL exponent array");
    if (int rc = settle(h)) return rc;
    for (int c = 0; c < 3; ++c) exps[c] = h->s16e[c];
    return LB_OK;
}

int lb_set_scales(lb_lattice *h, const int *exps)
{
    if (int rc = check(h)) return rc;
    if (h->codec != kS16) return fail(LB_EINVAL, "scales exist for LB_S16 storage only");
    if (!exps) return fail(LB_EINVAL, "NULL exponent array");
    for (int c = 0; c < 3; ++c)
        if (exps[c] < kS16MinExp || exps[c] > kS16MaxExp)
            return fail(LB_EINVAL, "exponent %d of weight class %d outside [%d, %d]", exps[c], c, kS16MinExp, kS16MaxExp);
    if (int rc = settle(h)) return rc;
    for (int c = 0; c < 3; ++c) h->s16e[c] = exps[c];
    s16_update_scales(h);
    return LB_OK;
}

long long lb_steps_done(const lb_lattice *h)
{
    if (!h || h->magic != kMagic) return -1;
    return h->steps;
}

long long lb_query(const lb_lattice *h, int key)
{
    if (!h || h->magic != kMagic) return -1;
    switch (key) {
        case 0: return h->variant;
        case 1: return h->vsites;
        case 2: return h->solids ? 1 : 0;
        case 3: return h->esize;
        case 4: return h->grid;
        case 5: return 1ll << h->lay.lg_r;
        case 6: return (long long)h->n_fluid;
        case 7: return (long long)(h->arr_elems * h->esize);
        case 8: return h->inplace ? 1 : 0;
        case 9: return h->codec;
        case 10: return h->rescales;
        case 11: return h->tile_order;
        case 12: return h->pull_nt;
        default: return -1;
    }
}

int lb_time_steps(lb_lattice *h, int n, double *ms)
{
    if (int rc = check(h)) return rc;
    if (n < 1 || !ms) return fail(LB_EINVAL, "n must be >= 1 and ms non-NULL");
    if (int rc = prepare_graphs(h, n)) return rc;
    Events evs(2);
    HIP_OR_FAIL(evs.create());
    hipEvent_t e0 = evs[0], e1 = evs[1];
    int rc = LB_OK;
    if (hipEventRecord(e0, h->stream) != hipSuccess) rc = fail(LB_EHIP, "hipEventRecord");
    if (rc == LB_OK) rc = enqueue_steps(h, n, nullptr, nullptr);
    // scaled storage: steps redone after a widening count in the timed region
    if (rc == LB_OK) rc = settle(h);
    if (rc == LB_OK && hipEventRecord(e1, h->stream) != hipSuccess) rc = fail(LB_EHIP, "hipEventRecord");
    if (rc == LB_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(LB_EHIP, "hipEventSynchronize");
    float t = 0.0f;
    if (rc == LB_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = fail(LB_EHIP, "hipEventElapsedTime");
    if (rc == LB_OK) *ms = t;
    return rc;
}

int lb_tune(lb_lattice *h, int reps)
{
    if (int rc = check(h)) return rc;
    if (reps < 1 || reps > 1000) return fail(LB_EINVAL, "reps must be in [1, 1000] (got %d)", reps);
    if (h->inplace) return fail(LB_EINVAL, "the in-place step has one launch shape per lattice");
    if (int rc = settle(h)) return rc;
    // candidates: vector widths that divide nx, each with both tile orders
    // and, with solids, both cache policies of the pulls (the force-field
    // kernels always pull with cached loads)
    struct Cand {
        int variant, order, grid, nt;
        double ms;
    };
    std::vector<Cand> cands;
    int max_grid = h->grid;
    for (int v = 1; v <= 3; ++v) {
        const int V = sites_per_thread(h->codec, v);
        if (h->nx % V != 0) continue;
        const uint64_t tiles = (h->n / V + kBlock - 1) / kBlock;
        if (tiles > 0x7fffffffull) continue;
        for (int order = 0; order < 3; ++order)
            for (int nt = 0; nt < (h->solids && !h->ffield ? 2 : 1); ++nt)
                cands.push_back(Cand{v, order, (int)tiles, nt, 0.0});
        max_grid = std::max(max_grid, (int)tiles);
    }
    if (cands.empty()) return LB_OK;  // only the one-site kernel fits this nx
    // partials for the largest grid (timing launches, and the choice)
    if (max_grid > h->grid) {
        HIP_OR_FAIL(hipStreamSynchronize(h->stream));
        (void)hipFree(h->partials);
        (void)hipFree(h->gpartials);
        h->partials = h->gpartials = nullptr;
        const size_t ngroups = ((size_t)max_grid + kRedChunk - 1) / kRedChunk;
        if (hipMalloc(&h->partials, (size_t)max_grid * 8 * sizeof(double)) != hipSuccess ||
            hipMalloc(&h->gpartials, ngroups * 4 * sizeof(double)) != hipSuccess)
            return fail(LB_ENOMEM, "hipMalloc(partials)");
    }
    // every timing launch reads the current state and writes the other array,
    // and, like a step inside a run, its first workgroup appends the totals
    // of the previous launch (the append's cost grows with the grid) -- into
    // a ring and counter of the tuner's own: the state, the step count and
    // the lattice's totals stay as they are
    double *tring = nullptr;
    unsigned long long *tctr = nullptr;
    if (hipMalloc(&tring, 64 * 4 * sizeof(double)) != hipSuccess ||
        hipMalloc(&tctr, sizeof(unsigned long long)) != hipSuccess) {
        if (tring) (void)hipFree(tring);
        return fail(LB_ENOMEM, "hipMalloc(tuner totals)");
    }
    Events evs(2);
    HIP_OR_FAIL(evs.create());
    const int saved_variant = h->variant, saved_order = h->tile_order, saved_nt = h->pull_nt;
    int rc = LB_OK;
    // two passes over the candidates, each keeping its faster timing (drift
    // of the clocks during the sweep then favours no candidate)
    for (Cand &c : cands) c.ms = 1e30;
    for (int pass = 0; pass < 2 && rc == LB_OK; ++pass)
    for (Cand &c : cands) {
        h->variant = c.variant;
        h->tile_order = c.order;
        h->pull_nt = c.nt;
        if (hipMemsetAsync(tctr, 0, sizeof(unsigned long long), h->stream) != hipSuccess) rc = fail(LB_EHIP, "memset");
        auto launch = [&](int k) {
            StepArgs a = step_args(h, h->cur, nullptr, nullptr, c.variant);
            a.partials = h->partials + (size_t)(k & 1) * 4 * c.grid;
            if (k > 0) {
                TotalsArgs t{};
                t.partials = h->partials + (size_t)((k - 1) & 1) * 4 * c.grid;
                t.nparts = c.grid;
                t.gpartials = h->gpartials;
                t.ring = tring;
                t.step_counter = tctr;
                t.n_fluid = h->n_fluid;
                a.prev = t;
            }
            if (launch_step(h->codec, c.variant, h->solids, false, a, c.grid, h->stream) != hipSuccess)
                rc = fail(LB_EHIP, "step kernel launch");
        };
        for (int k = 0; k < 2 && rc == LB_OK; ++k) launch(k);  // warm-up
        if (rc == LB_OK && hipEventRecord(evs[0], h->stream) != hipSuccess) rc = fail(LB_EHIP, "hipEventRecord");
        for (int k = 2; k < reps + 2 && rc == LB_OK; ++k) launch(k);
        if (rc == LB_OK && hipEventRecord(evs[1], h->stream) != hipSuccess) rc = fail(LB_EHIP, "hipEventRecord");
        float t = 0.0f;
        if (rc == LB_OK && hipEventSynchronize(evs[1]) != hipSuccess) rc = fail(LB_EHIP, "hipEventSynchronize");
        if (rc == LB_OK && hipEventElapsedTime(&t, evs[0], evs[1]) != hipSuccess) rc = fail(LB_EHIP, "hipEventElapsedTime");
        c.ms = std::min(c.ms, (double)t / reps);
        if (rc != LB_OK) break;
    }
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(tring);
    (void)hipFree(tctr);
    h->variant = saved_variant;
    h->tile_order = saved_order;
    h->pull_nt = saved_nt;
    if (rc != LB_OK) return rc;
    const Cand *best = &cands[0];
    for (const Cand &c : cands)
        if (c.ms < best->ms) best = &c;
    h->variant = best->variant;
    h->vsites = sites_per_thread(h->codec, best->variant);
    h->tile_order = best->order;
    h->pull_nt = best->nt;
    h->grid = best->grid;
    h->graphs.invalidate();
    if (h->codec == kS16) HIP_OR_FAIL(launch_zero_words(h->ovf, 2, h->stream));  // timing launches may flag
    HIP_OR_FAIL(hipStreamSynchronize(h->stream));
    return LB_OK;
}

int lb_time_step_kernel(lb_lattice *h, int n, double *ms)
{
    if (int rc = check(h)) return rc;
    if (n < 1 || !ms) return fail(LB_EINVAL, "n must be >= 1 and ms non-NULL");
    std::vector<hipEvent_t> ev(2 * (size_t)n, nullptr);
    int rc = LB_OK;
    for (auto &e : ev)
        if (rc == LB_OK && hipEventCreate(&e) != hipSuccess) rc = fail(LB_EHIP, "hipEventCreate");
    for (int k = 0; k < n && rc == LB_OK; ++k) {
        StepArgs a = step_args(h, h->cur, nullptr, nullptr);
        if (hipEventRecord(ev[2 * k], h->stream) != hipSuccess) rc = fail(LB_EHIP, "hipEventRecord");
        const hipError_t le = h->inplace ? launch_aa_step(h->codec, h->variant, h->solids, h->cur == 0, a, h->grid, h->stream)
                                         : launch_step(h->codec, h->variant, h->solids, false, a, h->grid, h->stream);
        if (rc == LB_OK && le != hipSuccess) rc = fail(LB_EHIP, "step kernel launch");
        if (rc == LB_OK && hipEventRecord(ev[2 * k + 1], h->stream) != hipSuccess) rc = fail(LB_EHIP, "hipEventRecord");
        if (rc == LB_OK && launch_totals(totals_args(h, 0, own_bufs(h), h->cur), h->stream) != hipSuccess) rc = fail(LB_EHIP, "totals launch");
        if (rc == LB_OK) {
            h->cur ^= 1;
            h->steps += 1;
        }
    }
    double total = 0.0;
    if (rc == LB_OK && hipEventSynchronize(ev[2 * n - 1]) != hipSuccess) rc = fail(LB_EHIP, "hipEventSynchronize");
    for (int k = 0; k < n && rc == LB_OK; ++k) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]) != hipSuccess) rc = fail(LB_EHIP, "hipEventElapsedTime");
        total += t;
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc == LB_OK) *ms = total / n;
    if (rc == LB_OK) rc = settle(h);
    return rc;
}

int lb_copy_probe(lb_lattice *h, int reps, double *ms)
{
    if (int rc = check(h)) return rc;
    if (reps < 1 || !ms) return fail(LB_EINVAL, "reps must be >= 1 and ms non-NULL");
    if (int rc = settle(h)) return rc;  // the probe overwrites the other array
    const uint64_t bytes = ((uint64_t)h->arr_elems * h->esize) & ~(uint64_t)15;
    Events evs(2);
    HIP_OR_FAIL(evs.create());
    hipEvent_t e0 = evs[0], e1 = evs[1];
    int rc = LB_OK;
    if (launch_copy(h->buf[h->cur], h->buf[h->cur ^ 1], bytes, h->stream) != hipSuccess)  // warm-up
        rc = fail(LB_EHIP, "copy kernel launch");
    if (rc == LB_OK && hipEventRecord(e0, h->stream) != hipSuccess) rc = fail(LB_EHIP, "hipEventRecord");
    for (int r = 0; r < reps && rc == LB_OK; ++r)
        if (launch_copy(h->buf[h->cur], h->buf[h->cur ^ 1], bytes, h->stream) != hipSuccess)
            rc = fail(LB_EHIP, "copy kernel launch");
    if (rc == LB_OK && hipEventRecord(e1, h->stream) != hipSuccess) rc = fail(LB_EHIP, "hipEventRecord");
    if (rc == LB_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(LB_EHIP, "hipEventSynchronize");
    float t = 0.0f;
    if (rc == LB_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = fail(LB_EHIP, "hipEventElapsedTime");
    if (rc == LB_OK) *ms = t / reps;
    return rc;
}

}  // extern "C"
