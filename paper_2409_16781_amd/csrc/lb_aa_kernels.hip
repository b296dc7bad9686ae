// In-place (one-array) storage: the two alternating step kernels.
#include "lb_device.h"

namespace lbm {
namespace {

// ------------------------------------------------------- in-place (AA) --
// One population array instead of two (the "AA" access pattern applied to
// the fused update of Section 3.1).  Two representations alternate:
//   even: slot opp(i) of site x holds S_i(x), the stored state, swapped;
//   odd:  slot i of site x holds f_i(x), the populations the next step
//         collides (already pulled, bounce-back included).
// From even, a step gathers f_i(x) = S_i(x - c_i) from slot opp(i) of x - c_i
// (its own slot i where x - c_i is solid), collides, and pushes f*_i(x) into
// slot i of x + c_i (its own slot opp(i) where x + c_i is solid).  From odd,
// a step reads slot i of x, collides and writes f*_i(x) into slot opp(i) of
// x.  Either way a site reads and writes the same 19 locations and no other
// site touches them, so the update is in place and needs no second array.
// The push shares x-edge elements between lanes through LDS, so tiles must
// hold whole rows (lds_edges).  Solid sites push nothing: their slots are the
// targets of their neighbours' bounce-back.

// Collide the V sites of a lane (FP32 arithmetic, storage codec C) exactly as
// the two-array step does; rho and u are not kept.
template <int C, int NW>
__device__ __forceinline__ void collide_lane(Lane<NW> (&d)[kQ], const Coll &cp)
{
    constexpr int V = NW * 4 / Codec<C>::kBytes;
    float mr[V], mu[V], mv[V], mw[V], fxs[V];
    Range16 rng;
    const Scale16 sc{};
    collide_sites<C, NW, false>(d, cp, sc, rng, fxs, mr, mu, mv, mw);
}

// Wave budget of the in-place kernels: that of the two-array step (the same
// collision code).
template <int C, int NW>
constexpr int aa_waves()
{
    return vec_waves<C, NW>();
}

// The lane's solid sites (bit e: site e is solid) and their neighbour masks.
template <int V, bool kSolids>
__device__ __forceinline__ uint32_t own_masks(const StepArgs &a, const TileGeom &g, uint32_t (&m)[V])
{
    uint32_t dead = 0;
#pragma unroll
    for (int e = 0; e < V; ++e) m[e] = 0;
    if constexpr (kSolids) {
        if (wave_dirty(a, g)) {
            load_masks<V>(a.nbmask + g.s0, m);
#pragma unroll
            for (int e = 0; e < V; ++e) dead |= (m[e] >> 31) << e;
        }
    }
    return dead;
}

// Odd -> even: read, collide, write swapped, all at the site itself.
template <int C, int NW, bool kSolids>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(aa_waves<C, NW>()))) void aa_local(StepArgs a)
{
    using K = Codec<C>;
    constexpr int V = NW * 4 / K::kBytes;
    char *F = reinterpret_cast<char *>(a.dst);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int ntiles = (a.nslots + kBlock - 1) / kBlock;
    if (const int b = blockIdx.x; b < ntiles) {  // one workgroup per tile
        const TileGeom g = tile_geom<V, false>(a, tile_of(b, ntiles, a.tile_order));
        Lane<NW> d[kQ];
#pragma unroll
        for (int i = 0; i < kQ; ++i) d[i] = ldv<NW>(F + (g.own + i * a.lay.seg) * K::kBytes);
        uint32_t m[V];
        const uint32_t dead = own_masks<V, kSolids>(a, g, m);
        collide_lane<C, NW>(d, a.coll);
        if (g.active) {
            if (dead) {
#pragma unroll
                for (int e = 0; e < V; ++e)
                    if ((dead >> e) & 1u) {
#pragma unroll
                        for (int i = 0; i < kQ; ++i) vset<C, NW>(d[i], e, 0u);
                    }
            }
            if (dead != (1u << V) - 1u) {
                const StoreBase sb = store_base(F, g.own, K::kBytes);
                if (dead == 0) {
#pragma unroll
                    for (int i = 0; i < kQ; ++i) stv_pop<NW>(sb, (uint32_t)OPP[i] * a.lay.seg * (uint32_t)K::kBytes, d[i]);
                } else {
#pragma unroll
                    for (int i = 0; i < kQ; ++i)
#pragma unroll
                        for (int e = 0; e < V; ++e)
                            if (!((dead >> e) & 1u)) st_elem<C>(F, g.own + OPP[i] * a.lay.seg + e, vget<C, NW>(d[i], e));
                }
            }
            add_lane_totals<C, NW>(d, acc, a.sc);
        }
    }
    store_block_totals(acc, a.partials + 4 * (size_t)blockIdx.x);
}

// Even -> odd: gather (transposed slots), collide, push to the neighbours.
// (The 16-bit codecs keep the three-wave budget of the two-array step: with
// two waves and no spills the kernel measured 10% slower at 512^3.)
// Wave budget of the push step: the FP16 push spills at three waves per SIMD
// (168 VGPRs) and runs faster at two (2.33 against 2.59 ms per 512^3 step);
// BF16 spills less and keeps three (1.83 ms).
template <int C, int NW>
constexpr int push_waves()
{
    return (C == kF16 && NW <= 2) ? 2 : aa_waves<C, NW>();
}

template <int C, int NW, bool kSolids>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(push_waves<C, NW>()))) void aa_pullpush(StepArgs a)
{
    using K = Codec<C>;
    constexpr int V = NW * 4 / K::kBytes;
    constexpr uint32_t kAll = (1u << V) - 1u;
    __shared__ EdgeLds lds;
    __shared__ uint32_t dead_row_last[kBlock], dead_row_first[kBlock], dead_wave_last[4], dead_wave_first[4];
    char *F = reinterpret_cast<char *>(a.dst);
    const uint32_t nx = (uint32_t)a.nx, ny = (uint32_t)a.ny, nz = (uint32_t)a.nz;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rit = (int)threadIdx.x >> a.lg_row_lanes;
    const int ntiles = (a.nslots + kBlock - 1) / kBlock;
    if (const int b = blockIdx.x; b < ntiles) {  // one workgroup per tile
        const TileGeom g = tile_geom<V, false>(a, tile_of(b, ntiles, a.tile_order));
        Lane<NW> d[kQ];
        const uint32_t dead = gather<C, NW, kSolids, false, true>(a, F, g, d, lds);
        uint32_t m[V];
        (void)own_masks<V, kSolids>(a, g, m);
        collide_lane<C, NW>(d, a.coll);
        if (dead) {
#pragma unroll
            for (int e = 0; e < V; ++e)
                if ((dead >> e) & 1u) {
#pragma unroll
                    for (int i = 0; i < kQ; ++i) vset<C, NW>(d[i], e, 0u);
                }
        }
        if (g.active) {
            add_lane_totals<C, NW>(d, acc, a.sc);
            // bounce-back: where x + c_i is solid (bit opp(i)), f*_i(x) stays at x, in slot opp(i)
            if constexpr (kSolids) {
#pragma unroll
                for (int i = 1; i < kQ; ++i)
#pragma unroll
                    for (int e = 0; e < V; ++e)
                        if (!((dead >> e) & 1u) && ((m[e] >> OPP[i]) & 1u))
                            st_elem<C>(F, g.own + OPP[i] * a.lay.seg + e, vget<C, NW>(d[i], e));
            }
        }
        // the pushed vector of direction i at positions x0..x0+V-1 of row
        // (y + c_iy, z + c_iz) holds f*_i of the sites x0 - c_ix .. of this row
        const uint32_t x0 = g.x0;
        const bool row_end = x0 + V >= nx;
        const bool left_edge = (lane == 0) || (x0 == 0);
        const bool right_edge = (lane == 63) || row_end;
        __syncthreads();  // the gather's readers of lds are done
        if (row_end) {
#pragma unroll
            for (int k = 0; k < 5; ++k) lds.row_last[rit][k] = d[kPlusX[k]].w[NW - 1];
            if constexpr (kSolids) dead_row_last[rit] = (dead >> (V - 1)) & 1u;
        }
        if (x0 == 0) {
#pragma unroll
            for (int k = 0; k < 5; ++k) lds.row_first[rit][k] = d[kMinusX[k]].w[0];
            if constexpr (kSolids) dead_row_first[rit] = dead & 1u;
        }
        if (lane == 63) {
#pragma unroll
            for (int k = 0; k < 5; ++k) lds.wave_last[wave][k] = d[kPlusX[k]].w[NW - 1];
            if constexpr (kSolids) dead_wave_last[wave] = (dead >> (V - 1)) & 1u;
        }
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 5; ++k) lds.wave_first[wave][k] = d[kMinusX[k]].w[0];
            if constexpr (kSolids) dead_wave_first[wave] = dead & 1u;
        }
        __syncthreads();
        // source-dead bits of the shifted vectors
        uint32_t dead_plus = dead, dead_minus = dead;
        if constexpr (kSolids) {
            uint32_t dp = (uint32_t)wave_shr1((dead >> (V - 1)) & 1u);
            if (left_edge) dp = x0 == 0 ? dead_row_last[rit] : dead_wave_last[wave - 1];
            dead_plus = ((dead << 1) | dp) & kAll;
            uint32_t dn = (uint32_t)wave_shl1(dead & 1u);
            if (right_edge) dn = row_end ? dead_row_first[rit] : dead_wave_first[wave + 1];
            dead_minus = (dead >> 1) | (dn << (V - 1));
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const int i = kPlusX[k];  // pushed to x + 1: position p holds site p - 1
            uint32_t prev = wave_shr1(d[i].w[NW - 1]);
            if (left_edge) prev = x0 == 0 ? lds.row_last[rit][k] : lds.wave_last[wave - 1][k];
            if constexpr (K::kBytes == 2) prev >>= 16;
            d[i] = shift_in_from_left<C, NW>(d[i], prev);
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const int i = kMinusX[k];  // pushed to x - 1: position p holds site p + 1
            uint32_t next = wave_shl1(d[i].w[0]);
            if (right_edge) next = row_end ? lds.row_first[rit][k] : lds.wave_first[wave + 1][k];
            if constexpr (K::kBytes == 2) next &= 0xffffu;
            d[i] = shift_in_from_right<C, NW>(d[i], next);
        }
        if (g.active) {
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const uint32_t ty = CY[i] > 0 ? g.yp : (CY[i] < 0 ? g.ym : g.y);
                const uint32_t tz = CZ[i] > 0 ? g.zp : (CZ[i] < 0 ? g.zm : g.z);
                const uint64_t t = a.lay.row_base(tz * ny + ty) + (uint64_t)i * a.lay.seg + x0;
                const uint32_t sd = CX[i] > 0 ? dead_plus : (CX[i] < 0 ? dead_minus : dead);
                if (sd == 0) {
                    // buffer stores (device-scope policy) when every target of
                    // the wave lies at or after the first active lane's, which
                    // fails only where the periodic wrap puts a later lane's
                    // target row first
                    const StoreBase sb = store_base(F, t, K::kBytes);
                    if (__builtin_amdgcn_ballot_w64(t >= sb.first) == __builtin_amdgcn_read_exec())
                        stv_at<NW>(F, sb, t, K::kBytes, d[i]);
                    else
                        stv<NW>(F + t * K::kBytes, d[i]);
                } else if (sd != kAll) {
#pragma unroll
                    for (int e = 0; e < V; ++e)
                        if (!((sd >> e) & 1u)) st_elem<C>(F, t + e, vget<C, NW>(d[i], e));
                }
            }
        }
        (void)nz;
    }
    store_block_totals(acc, a.partials + 4 * (size_t)blockIdx.x);
}

}  // namespace

namespace {
template <int C, int NW, bool S>
void *aa_fn(bool from_even)
{
    return from_even ? reinterpret_cast<void *>(&aa_pullpush<C, NW, S>) : reinterpret_cast<void *>(&aa_local<C, NW, S>);
}
template <int C, bool S>
void *aa_pick_nw(int variant, bool from_even)
{
    if (variant == 1) return aa_fn<C, 4, S>(from_even);
    if (variant == 2) return aa_fn<C, 2, S>(from_even);
    return aa_fn<C, 1, S>(from_even);
}
void *pick_aa(int codec, int variant, bool solids, bool from_even)
{
    switch (codec) {
        case kF32: return solids ? aa_pick_nw<kF32, true>(variant, from_even) : aa_pick_nw<kF32, false>(variant, from_even);
        case kF16: return solids ? aa_pick_nw<kF16, true>(variant, from_even) : aa_pick_nw<kF16, false>(variant, from_even);
        default: return solids ? aa_pick_nw<kBF16, true>(variant, from_even) : aa_pick_nw<kBF16, false>(variant, from_even);
    }
}
}  // namespace

hipError_t launch_aa_step(int codec, int variant, bool solids, bool from_even, const StepArgs &a, int grid,
                          hipStream_t s)
{
    StepArgs arg = a;
    void *params[] = {&arg};
    return hipLaunchKernel(pick_aa(codec, variant, solids, from_even), dim3(grid), dim3(kBlock), params, 0, s);
}

int aa_occupancy(int codec, int variant, bool solids, bool from_even)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pick_aa(codec, variant, solids, from_even), kBlock, 0) !=
        hipSuccess)
        return 1;
    return nb < 1 ? 1 : nb;
}

}  // namespace lbm
