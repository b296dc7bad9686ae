// Batch of lattices: the tiles of all domains in one launch per step, and
// the per-domain FP64 totals.
#include "lb_device.h"

namespace lbm {
namespace {

// One step of a batch of lattices: the tiles of all domains in one launch.
// The domain table is read through the constant address space, so the
// per-tile domain parameters (uniform per workgroup) come in with scalar
// loads and live in scalar registers.
typedef LB_CONSTANT_AS const DomDesc ConstDomDesc;
typedef LB_CONSTANT_AS const int ConstInt;

// The per-domain totals of one batch step from its tile partials, summed by
// one workgroup exactly as reduce_domains does and appended to the rings.
// The partials come from an earlier launch: no fence is needed.
__device__ __forceinline__ void append_batch_totals(const BatchTotalsArgs &t)
{
    const unsigned long long step = __hip_atomic_load(t.step_counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // the four waves take domains in turn, each sum in reduce_domains' order
    for (int d = (int)threadIdx.x >> 6; d < t.ndoms; d += kBlock / 64) {
        const DomDesc &D = t.doms[d];
        double tot[4];
        wave_sum4(t.partials + 4 * (size_t)D.tile_begin, D.ntiles, tot);
        if ((threadIdx.x & 63) == 0) {
            double *r = t.ring + 4 * ((size_t)d * kRingCap + step % kRingCap);
            r[0] = D.n_fluid + tot[0];
            r[1] = tot[1];
            r[2] = tot[2];
            r[3] = tot[3];
        }
    }
    if (threadIdx.x == 0) __hip_atomic_store(t.step_counter, step + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int C, int NW>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(vec_waves<C, NW>()))) void step_batch(BatchArgs a)
{
    __shared__ EdgeLds lds;
    for (int b = blockIdx.x; b < a.ntiles; b += gridDim.x) {
        const int t = tile_of(b, a.ntiles, a.tile_order);
        const int dom = ((ConstInt *)a.tile_dom)[t];
        ConstDomDesc &D = ((ConstDomDesc *)a.doms)[dom];
        const StepArgs s = D.s;
        const char *src = reinterpret_cast<const char *>(D.buf[a.parity]);
        char *dst = reinterpret_cast<char *>(D.buf[a.parity ^ 1]);
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        tile_update<C, NW, true, false, true>(s, src, dst, t - D.tile_begin, acc, lds);
        store_block_totals(acc, a.partials + 4 * (size_t)t);
        __syncthreads();  // the totals' LDS is reused by the next tile
    }
    if (a.prev.partials != nullptr && blockIdx.x == 0) append_batch_totals(a.prev);
}

// Per-domain totals of a batch step: workgroup d sums the partials of domain
// d's tiles in order and stores {mass, momentum} in the domain's ring; the
// last workgroup to finish advances the step counter.
__global__ __launch_bounds__(kBlock) void reduce_domains(BatchTotalsArgs a)
{
    __shared__ int is_last;
    const int d = blockIdx.x;
    const unsigned long long step = __hip_atomic_load(a.step_counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    double tot[4];
    block_sum4(a.partials + 4 * (size_t)a.doms[d].tile_begin, a.doms[d].ntiles, tot, false);
    if (threadIdx.x == 0) {
        double *r = a.ring + 4 * ((size_t)d * kRingCap + step % kRingCap);
        r[0] = a.doms[d].n_fluid + tot[0];
        r[1] = tot[1];
        r[2] = tot[2];
        r[3] = tot[3];
        __threadfence();
        const unsigned int prev = atomicAdd(a.ticket, 1u);
        is_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (is_last && threadIdx.x == 0) {
        __hip_atomic_store(a.step_counter, step + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(a.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace

namespace {
template <int C>
void *batch_fn(int variant)
{
    if (variant == 1) return reinterpret_cast<void *>(&step_batch<C, 4>);
    if (variant == 2) return reinterpret_cast<void *>(&step_batch<C, 2>);
    return reinterpret_cast<void *>(&step_batch<C, 1>);
}

void *pick_batch(int codec, int variant)
{
    switch (codec) {
        case kF32: return batch_fn<kF32>(variant);
        case kF16: return batch_fn<kF16>(variant);
        default: return batch_fn<kBF16>(variant);
    }
}
}  // namespace

hipError_t launch_batch_step(int codec, int variant, const BatchArgs &a, int grid, size_t lds_pad, hipStream_t s)
{
    BatchArgs arg = a;
    void *params[] = {&arg};
    return hipLaunchKernel(pick_batch(codec, variant), dim3(grid), dim3(kBlock), params, lds_pad, s);
}

size_t batch_cap_lds(int codec, int variant, int wg_cap)
{
    if (wg_cap <= 0) return 0;
    hipFuncAttributes at;
    int dev = 0, lds_cu = 0;
    if (hipFuncGetAttributes(&at, pick_batch(codec, variant)) != hipSuccess || hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess)
        return 0;
    // wg_cap + 1 workgroups of (static + pad) bytes must not fit in a CU's LDS
    const size_t per = (size_t)lds_cu / (size_t)(wg_cap + 1) + 1;
    return per > at.sharedSizeBytes ? per - at.sharedSizeBytes : 0;
}

hipError_t launch_batch_totals(const BatchTotalsArgs &a, hipStream_t s)
{
    reduce_domains<<<a.ndoms, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

int batch_occupancy(int codec, int variant, size_t lds_pad)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pick_batch(codec, variant), kBlock, lds_pad) != hipSuccess)
        return 1;
    return nb < 1 ? 1 : nb;
}

}  // namespace lbm
