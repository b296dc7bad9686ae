// Host runtime of two-dimensional D2Q9 lattices (declared in include/lb.h):
// the paper's own model and lid-driven cavity workload (Sections 2 and 3.3),
// run by the same fused pull update as the D3Q19 lattices, FP32 storage of
// f - w, two arrays swapped by parity, FP64 totals per step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "lb.h"
#include "lb_host.h"
#include "lb_internal.h"

using namespace lbm;

namespace {
constexpr uint64_t kMagic2 = 0x4c42443251392121ull;  // "LBD2Q9!!"
constexpr uint64_t kDead2 = 0xdead2d9adead2d9aull;
}  // namespace

struct lb2d_lattice {
    uint64_t magic = 0;
    int nx = 0, ny = 0;
    uint64_t n = 0;
    double tau = 0, omega = 0, lid[2] = {0, 0};
    Layout lay{};
    uint64_t arr_elems = 0;
    void *buf[2] = {nullptr, nullptr};
    int cur = 0;
    uint8_t *flags = nullptr;
    uint32_t *nbmask = nullptr;
    uint8_t *chunkdirty = nullptr;  // one byte per 64 sites
    bool solids = false;
    double n_fluid = 0;
    double *partials = nullptr, *gpartials = nullptr, *ring = nullptr;
    unsigned int *ticket = nullptr;
    unsigned long long *counter = nullptr;
    hipStream_t stream = nullptr;
    int variant = 1, vsites = 4, grid = 1;
    long long steps = 0;
};

namespace {

int check2(const lb2d_lattice *h)
{
    if (!h || h->magic != kMagic2) return fail(LB_ESTATE, "invalid or destroyed D2Q9 lattice handle");
    return LB_OK;
}

void release2(lb2d_lattice *h)
{
    void *p[] = {h->buf[0], h->buf[1], h->flags, h->nbmask, h->chunkdirty, h->partials, h->gpartials, h->ring,
                 h->ticket, h->counter};
    for (void *q : p)
        if (q) (void)hipFree(q);
}

Step2Args step2_args(const lb2d_lattice *h, int from)
{
    Step2Args a{};
    a.src = h->buf[from];
    a.dst = h->buf[from ^ 1];
    a.lay = h->lay;
    a.nx = h->nx;
    a.ny = h->ny;
    a.nslots = (int)(h->n / (uint64_t)h->vsites);
    const int row_lanes = h->nx / h->vsites;
    a.lds_edges = (row_lanes <= kBlock && kBlock % row_lanes == 0) ? 1 : 0;
    a.lg_row_lanes = 0;
    while ((1 << a.lg_row_lanes) < row_lanes) ++a.lg_row_lanes;
    a.div_pitch = make_fastdiv((uint32_t)h->nx);
    const float om = (float)h->omega;
    a.hom = 0.5f * om;
    a.ow1 = om * (1.0f / 9.0f);
    a.ow2 = om * (1.0f / 36.0f);
    a.q1 = 4.5f * om * (1.0f / 9.0f);
    a.q2 = 4.5f * om * (1.0f / 36.0f);
    const int cx[9] = {0, 1, -1, 0, 0, 1, 1, -1, -1}, cy[9] = {0, 0, 0, 1, -1, 1, -1, 1, -1};
    for (int i = 0; i < 9; ++i) {
        const double w = i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
        a.lidc[i] = (float)(6.0 * w * (cx[i] * h->lid[0] + cy[i] * h->lid[1]));
    }
    a.nbmask = h->nbmask;
    a.chunkdirty = h->chunkdirty;
    a.partials = h->partials;
    return a;
}

// Totals of the step whose workgroup partials are in buffer buf (0 or 1).
TotalsArgs totals2(const lb2d_lattice *h, int buf)
{
    TotalsArgs t{};
    t.partials = h->partials + (size_t)buf * 4 * h->grid;
    t.nparts = h->grid;
    t.gpartials = h->gpartials;
    t.ticket = h->ticket;
    t.ring = h->ring;
    t.step_counter = h->counter;
    t.n_fluid = h->n_fluid;
    return t;
}

// n steps as one run: step k writes its workgroup partials into buffer k & 1
// and the first workgroup of step k + 1 appends the totals of step k; one
// totals kernel closes the run (the ring holds the same values as with one
// totals kernel per step).
int enqueue2(lb2d_lattice *h, int n)
{
    for (int k = 0; k < n; ++k) {
        Step2Args a = step2_args(h, h->cur);
        a.partials = h->partials + (size_t)(k & 1) * 4 * h->grid;
        if (k > 0) a.prev = totals2(h, (k - 1) & 1);
        HIP_OR_FAIL(launch_step2d(h->variant, h->solids, a, h->grid, h->stream));
        h->cur ^= 1;
        h->steps += 1;
    }
    if (n > 0) HIP_OR_FAIL(launch_totals(totals2(h, (n - 1) & 1), h->stream));
    return LB_OK;
}

}  // namespace

extern "C" {

lb2d_lattice *lb2d_create(int nx, int ny, double tau, const uint8_t *flags, double lid_ux, double lid_uy,
                          void *hip_stream)
{
    if (nx < 1 || ny < 1 || (uint64_t)nx * ny > 0x7fffffffull - 4096) {
        fail(LB_EINVAL, "D2Q9 extents must be >= 1 with nx * ny < 2^31 - 4096 (got %d x %d)", nx, ny);
        return nullptr;
    }
    if (!(tau > 0.5)) {
        fail(LB_EINVAL, "tau must be > 0.5 or +inf (got %g)", tau);
        return nullptr;
    }
    if (!std::isfinite(lid_ux) || !std::isfinite(lid_uy)) {
        fail(LB_EINVAL, "the lid velocity must be finite");
        return nullptr;
    }
    const uint64_t n = (uint64_t)nx * ny;
    uint64_t nsolid = 0;
    if (flags) {
        for (uint64_t s = 0; s < n; ++s) {
            if (flags[s] > 2) {
                fail(LB_EINVAL, "flag value %d at site %llu (allowed: 0 fluid, 1 wall, 2 lid)", (int)flags[s],
                     (unsigned long long)s);
                return nullptr;
            }
            nsolid += flags[s] ? 1 : 0;
        }
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        fail(LB_EHIP, "no HIP device available");
        return nullptr;
    }
    lb2d_lattice *h = new (std::nothrow) lb2d_lattice();
    if (!h) {
        fail(LB_ENOMEM, "host allocation failed");
        return nullptr;
    }
    h->nx = nx;
    h->ny = ny;
    h->n = n;
    h->tau = tau;
    h->omega = std::isinf(tau) ? 0.0 : 1.0 / tau;
    h->lid[0] = lid_ux;
    h->lid[1] = lid_uy;
    h->stream = static_cast<hipStream_t>(hip_stream);
    h->solids = nsolid > 0;
    h->n_fluid = (double)(n - nsolid);
    // 16-byte vectors (4 sites per lane) when nx allows, else 8- or 4-byte
    h->variant = nx % 4 == 0 ? 1 : (nx % 2 == 0 ? 2 : 3);
    const long kv = env_long("LB_KERNEL2D", 0);
    if (kv >= 1 && kv <= 3 && nx % (kv == 1 ? 4 : (kv == 2 ? 2 : 1)) == 0) h->variant = (int)kv;
    h->vsites = h->variant == 1 ? 4 : (h->variant == 2 ? 2 : 1);
    // rows of 32 KiB blocks, as for the D3Q19 arrays
    uint64_t R = 1;
    while ((R * 2) * nx * 4 <= 32768 && R < (uint64_t)ny) R *= 2;
    uint32_t lg = 0;
    while ((1ull << lg) < R) ++lg;
    h->lay.nx = h->lay.pitch = (uint32_t)nx;
    h->lay.lg_r = lg;
    if (!block_fits((uint64_t)R * nx, 9, 4)) {
        delete h;
        fail(LB_EINVAL, "rows of %d sites are too long", nx);
        return nullptr;
    }
    h->lay.seg = (uint32_t)(R * nx);
    h->lay.blk = 9 * h->lay.seg;
    h->arr_elems = ((uint64_t)ny + R - 1) / R * h->lay.blk;
    const uint64_t tiles = (n / h->vsites + kBlock - 1) / kBlock;
    h->grid = (int)std::min<uint64_t>(tiles, 0x7fffffffull);  // one workgroup per tile

    auto bail = [&](int code, const char *what, hipError_t e) -> lb2d_lattice * {
        release2(h);
        delete h;
        fail(code, "%s: %s", what, hipGetErrorString(e));
        return nullptr;
    };
    const size_t bytes = (size_t)h->arr_elems * 4;
    hipError_t e;
    for (int b = 0; b < 2; ++b) {
        if ((e = hipMalloc(&h->buf[b], bytes)) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc(populations)", e);
        if ((e = hipMemsetAsync(h->buf[b], 0, bytes, h->stream)) != hipSuccess) return bail(LB_EHIP, "hipMemsetAsync", e);
    }
    const size_t ngroups = ((size_t)h->grid + kRedChunk - 1) / kRedChunk;
    if ((e = hipMalloc(&h->partials, (size_t)h->grid * 8 * sizeof(double))) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc", e);
    if ((e = hipMalloc(&h->gpartials, ngroups * 4 * sizeof(double))) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc", e);
    if ((e = hipMalloc(&h->ring, (size_t)kRingCap * 4 * sizeof(double))) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc", e);
    if ((e = hipMalloc(&h->ticket, sizeof(unsigned int))) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc", e);
    if ((e = hipMalloc(&h->counter, sizeof(unsigned long long))) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc", e);
    if ((e = hipMemsetAsync(h->ticket, 0, sizeof(unsigned int), h->stream)) != hipSuccess) return bail(LB_EHIP, "hipMemsetAsync", e);
    if ((e = hipMemsetAsync(h->counter, 0, sizeof(unsigned long long), h->stream)) != hipSuccess) return bail(LB_EHIP, "hipMemsetAsync", e);
    if ((e = hipMemsetAsync(h->ring, 0, (size_t)kRingCap * 4 * sizeof(double), h->stream)) != hipSuccess) return bail(LB_EHIP, "hipMemsetAsync", e);
    if (h->solids) {
        if ((e = hipMalloc(&h->flags, n)) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc(flags)", e);
        if ((e = hipMalloc(&h->nbmask, n * sizeof(uint32_t) + 64)) != hipSuccess) return bail(LB_ENOMEM, "hipMalloc(masks)", e);
        if ((e = hipMalloc(&h->chunkdirty, (size_t)(n + 63) / 64)) != hipSuccess)
            return bail(LB_ENOMEM, "hipMalloc(chunks)", e);
        if ((e = hipMemcpyAsync(h->flags, flags, n, hipMemcpyHostToDevice, h->stream)) != hipSuccess)
            return bail(LB_EHIP, "flags upload", e);
        if ((e = launch_masks2d(h->flags, nx, ny, h->nbmask, h->chunkdirty, h->stream)) != hipSuccess)
            return bail(LB_EHIP, "mask kernels", e);
    }
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return bail(LB_EHIP, "hipStreamSynchronize", e);
    h->magic = kMagic2;
    return h;
}

void lb2d_destroy(lb2d_lattice *h)
{
    if (!h || h->magic != kMagic2) return;
    (void)hipStreamSynchronize(h->stream);
    h->magic = kDead2;
    release2(h);
    delete h;
}

int lb2d_init_eq(lb2d_lattice *h, const double *rho, const double *u)
{
    if (int rc = check2(h)) return rc;
    HIP_OR_FAIL(launch_init2d(h->buf[0], h->lay, h->nx, h->ny, rho, u, h->flags, h->stream));
    HIP_OR_FAIL(hipMemsetAsync(h->counter, 0, sizeof(unsigned long long), h->stream));
    h->cur = 0;
    h->steps = 0;
    return LB_OK;
}

int lb2d_step(lb2d_lattice *h, int n)
{
    if (int rc = check2(h)) return rc;
    if (n < 0) return fail(LB_EINVAL, "step count must be >= 0 (got %d)", n);
    return enqueue2(h, n);
}

int lb2d_macros(lb2d_lattice *h, float *rho, float *u)
{
    if (int rc = check2(h)) return rc;
    HIP_OR_FAIL(launch_macros2d(h->buf[h->cur], h->lay, h->nx, h->ny, h->flags, rho, u, h->stream));
    return LB_OK;
}

int lb2d_sums(lb2d_lattice *h, double *out, int k)
{
    if (int rc = check2(h)) return rc;
    if (k < 1 || k > kRingCap || k > h->steps) return fail(LB_EINVAL, "k must be in [1, min(steps, %d)]", kRingCap);
    if (!out) return fail(LB_EINVAL, "NULL output");
    HIP_OR_FAIL(hipStreamSynchronize(h->stream));
    unsigned long long done = 0;
    HIP_OR_FAIL(hipMemcpy(&done, h->counter, sizeof done, hipMemcpyDeviceToHost));
    std::vector<double> ring((size_t)kRingCap * 4);
    HIP_OR_FAIL(hipMemcpy(ring.data(), h->ring, ring.size() * sizeof(double), hipMemcpyDeviceToHost));
    bool bad = false;
    for (int j = 0; j < k; ++j) {
        const unsigned long long st = done - (unsigned long long)k + j;
        for (int c = 0; c < 3; ++c) {
            out[3 * j + c] = ring[4 * (st % kRingCap) + c];
            if (!std::isfinite(out[3 * j + c])) bad = true;
        }
    }
    if (bad) return fail(LB_EUNSTABLE, "non-finite mass or momentum total");
    return LB_OK;
}

static int copy2(lb2d_lattice *h, void *buf, size_t bytes, int where, bool to_lattice)
{
    if (int rc = check2(h)) return rc;
    const size_t want = (size_t)9 * h->n * 4;
    if (bytes != want) return fail(LB_EINVAL, "buffer is %zu bytes, expected %zu", bytes, want);
    if (!buf) return fail(LB_EINVAL, "NULL buffer");
    if (where != LB_HOST && where != LB_DEVICE) return fail(LB_EINVAL, "where must be LB_HOST or LB_DEVICE");
    void *planes = buf;
    hipError_t e = hipSuccess;
    if (where == LB_HOST) {
        if ((e = hipMalloc(&planes, bytes)) != hipSuccess) return fail(LB_ENOMEM, "hipMalloc(staging)");
        if (to_lattice) e = hipMemcpyAsync(planes, buf, bytes, hipMemcpyHostToDevice, h->stream);
    }
    if (e == hipSuccess) e = launch_repack2d(planes, h->buf[h->cur], h->lay, (int64_t)h->n, to_lattice, h->stream);
    if (e == hipSuccess && where == LB_HOST && !to_lattice)
        e = hipMemcpyAsync(buf, planes, bytes, hipMemcpyDeviceToHost, h->stream);
    if (where == LB_HOST) {
        const hipError_t se = hipStreamSynchronize(h->stream);
        (void)hipFree(planes);
        if (e == hipSuccess) e = se;
    }
    if (e != hipSuccess) return fail(LB_EHIP, "population copy: %s", hipGetErrorString(e));
    return LB_OK;
}

int lb2d_get_f(lb2d_lattice *h, void *buf, size_t bytes, int where) { return copy2(h, buf, bytes, where, false); }

int lb2d_set_f(lb2d_lattice *h, const void *buf, size_t bytes, int where)
{
    return copy2(h, const_cast<void *>(buf), bytes, where, true);
}

int lb2d_sync(lb2d_lattice *h)
{
    if (int rc = check2(h)) return rc;
    HIP_OR_FAIL(hipStreamSynchronize(h->stream));
    return LB_OK;
}

long long lb2d_steps_done(lb2d_lattice *h)
{
    if (check2(h)) return -1;
    return h->steps;
}

int lb2d_time_steps(lb2d_lattice *h, int n, double *ms)
{
    if (int rc = check2(h)) return rc;
    if (n < 1 || !ms) return fail(LB_EINVAL, "n >= 1 and a result pointer are required");
    Events evs(2);
    HIP_OR_FAIL(evs.create());
    hipEvent_t e0 = evs[0], e1 = evs[1];
    int rc = LB_OK;
    if (hipEventRecord(e0, h->stream) != hipSuccess) rc = fail(LB_EHIP, "hipEventRecord");
    if (rc == LB_OK) rc = enqueue2(h, n);
    if (rc == LB_OK && hipEventRecord(e1, h->stream) != hipSuccess) rc = fail(LB_EHIP, "hipEventRecord");
    float t = 0.0f;
    if (rc == LB_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(LB_EHIP, "hipEventSynchronize");
    if (rc == LB_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = fail(LB_EHIP, "hipEventElapsedTime");
    if (rc == LB_OK) *ms = t;
    return rc;
}

}  // extern "C"
