// Two-dimensional D2Q9 lattices: step, masks, initialisation, macros and
// raw-state repacking.
#include "lb_device.h"

namespace lbm {
namespace {

// ----------------------------------------------------------- D2Q9 (2-D) --
// The paper's own two-dimensional model (D2Q9, Section 2 and Fig. 1) for the
// lid-driven cavity it benchmarks (Section 3.3): the same fused pull update,
// 9 populations, FP32 storage of f - w.  Bounce-back off a wall returns the
// site's own opposite value; off the lid it adds 6 w_i (c_i . u_lid).

constexpr int kQ2 = 9;
constexpr int CX2[kQ2] = {0, 1, -1, 0, 0, 1, 1, -1, -1};
constexpr int CY2[kQ2] = {0, 0, 0, 1, -1, 1, -1, 1, -1};
constexpr int OPP2[kQ2] = {0, 2, 1, 4, 3, 8, 7, 6, 5};
constexpr int kPlusX2[3] = {1, 5, 6};
constexpr int kMinusX2[3] = {2, 7, 8};

// BGK collision of one D2Q9 site (shifted populations, no force), written as
// pair increments like the D3Q19 collision: axis pairs (1,2), (3,4) take the
// remainder of sum_p c_p n_p = 0, the rest population that of the mass.
__device__ __forceinline__ void collide2(float (&g)[kQ2], const Step2Args &p, float &mass, float &px, float &py)
{
    const float s1 = g[1] + g[2], d1 = g[1] - g[2];
    const float s3 = g[3] + g[4], d3 = g[3] - g[4];
    const float s5 = g[5] + g[8], d5 = g[5] - g[8];
    const float s6 = g[6] + g[7], d6 = g[6] - g[7];
    const float drho = g[0] + (s1 + s3) + (s5 + s6);
    const float jx = d1 + d5 + d6;
    const float jy = d3 + d5 - d6;
    const float inv = __builtin_amdgcn_rcpf(1.0f + drho);
    const float ux = jx * inv, uy = jy * inv;
    const float t = drho - 1.5f * (jx * ux + jy * uy);
    const float base1 = p.ow1 * t, base2 = p.ow2 * t;
    const float c5 = jx + jy, c6 = jx - jy;
    constexpr float kSixth = 1.0f / 6.0f;
    const float n5 = d5 - kSixth * c5, n6 = d6 - kSixth * c6;
    const float n1 = -(n5 + n6), n3 = -(n5 - n6);
    float sum_hs = 0.0f;
    relax_pair(g[1], g[2], s1, n1, jx, inv, base1, p.q1, 0.0f, 0.0f, p.hom, sum_hs);
    relax_pair(g[3], g[4], s3, n3, jy, inv, base1, p.q1, 0.0f, 0.0f, p.hom, sum_hs);
    relax_pair(g[5], g[8], s5, n5, c5, inv, base2, p.q2, 0.0f, 0.0f, p.hom, sum_hs);
    relax_pair(g[6], g[7], s6, n6, c6, inv, base2, p.q2, 0.0f, 0.0f, p.hom, sum_hs);
    g[0] = g[0] - 2.0f * sum_hs;
    mass = drho;
    px = jx;
    py = jy;
}

template <int NW, bool kSolids>
__global__ __launch_bounds__(kBlock) void step2d(Step2Args a)
{
    using K = Codec<kF32>;
    constexpr int V = NW;
    __shared__ EdgeLds lds;
    const char *src = reinterpret_cast<const char *>(a.src);
    char *dst = reinterpret_cast<char *>(a.dst);
    const uint32_t nx = (uint32_t)a.nx, ny = (uint32_t)a.ny;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rit = (int)threadIdx.x >> a.lg_row_lanes;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int ntiles = (a.nslots + kBlock - 1) / kBlock;
    if (const int b = blockIdx.x; b < ntiles) {  // one workgroup per tile
        const int slot = b * kBlock + (int)threadIdx.x;
        const bool active = slot < a.nslots;
        const uint32_t s0 = (uint32_t)(active ? slot : a.nslots - 1) * V;
        const uint32_t y = fastdiv(s0, a.div_pitch);
        const uint32_t x0 = s0 - y * nx;
        const uint32_t ym = (y == 0 ? ny : y) - 1, yp = (y + 1 == ny) ? 0 : y + 1;
        const uint64_t own = a.lay.row_base(y) + x0;
        uint64_t rb[kQ2];
#pragma unroll
        for (int i = 0; i < kQ2; ++i)
            rb[i] = a.lay.row_base(CY2[i] > 0 ? ym : (CY2[i] < 0 ? yp : y)) + (uint64_t)i * a.lay.seg;
        bool dirty = false;  // the V sites share one 64-site chunk (V | 64)
        if constexpr (kSolids) dirty = a.chunkdirty[s0 >> 6] != 0;
        Lane<NW> d[kQ2];
#pragma unroll
        for (int i = 0; i < kQ2; ++i) d[i] = ldv<NW>(src + (rb[i] + x0) * 4);
        // Near solids: the masks and the site's own values of every population
        // that may bounce, loaded together with the pulls (not after the
        // masks).  Rows y +- 1 are not the own row, so directions 3..8 load
        // their opposite at the own row; for 1 and 2 it is the unshifted pull.
        uint32_t m[V];
        Lane<NW> ownv[kQ2];
        if constexpr (kSolids) {
            if (dirty) {
                load_masks<V>(a.nbmask + s0, m);
#pragma unroll
                for (int i = 3; i < kQ2; ++i) ownv[i] = ldv<NW>(src + (own + OPP2[i] * a.lay.seg) * 4);
            }
            ownv[1] = d[2];
            ownv[2] = d[1];
        }

        // x-edges: the element beyond a wave comes from the neighbouring
        // wave through LDS when that wave is in this tile and the element is
        // in the same row; the periodic wrap too when tiles hold whole rows;
        // anything else (tile ends of long rows) by a direct load
        const bool left_edge = (lane == 0) || (x0 == 0);
        const bool row_end = x0 + V >= nx;
        const bool right_edge = (lane == 63) || row_end;
        __syncthreads();  // the previous tile's readers of lds are done
        if (a.lds_edges) {
            if (row_end) {
#pragma unroll
                for (int k = 0; k < 3; ++k) lds.row_last[rit][k] = d[kPlusX2[k]].w[NW - 1];
            }
            if (x0 == 0) {
#pragma unroll
                for (int k = 0; k < 3; ++k) lds.row_first[rit][k] = d[kMinusX2[k]].w[0];
            }
        }
        if (lane == 63) {
#pragma unroll
            for (int k = 0; k < 3; ++k) lds.wave_last[wave][k] = d[kPlusX2[k]].w[NW - 1];
        }
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 3; ++k) lds.wave_first[wave][k] = d[kMinusX2[k]].w[0];
        }
        __syncthreads();
        const uint32_t xl = (x0 == 0 ? nx : x0) - 1;
        const uint32_t xr = row_end ? 0 : x0 + V;
        // the neighbour of a wave seam inside a row is a lane of this tile
        const bool left_lds = x0 == 0 ? a.lds_edges != 0 : wave > 0;
        const bool right_lds = row_end ? a.lds_edges != 0 : wave < kBlock / 64 - 1;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int i = kPlusX2[k];
            uint32_t prev = wave_shr1(d[i].w[NW - 1]);
            if (left_edge) prev = left_lds ? (x0 == 0 ? lds.row_last[rit][k] : lds.wave_last[wave - 1][k])
                                           : ld_elem<kF32>(src, rb[i] + xl);
            d[i] = shift_in_from_left<kF32, NW>(d[i], prev);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int i = kMinusX2[k];
            uint32_t next = wave_shl1(d[i].w[0]);
            if (right_edge) next = right_lds ? (row_end ? lds.row_first[rit][k] : lds.wave_first[wave + 1][k])
                                             : ld_elem<kF32>(src, rb[i] + xr);
            d[i] = shift_in_from_right<kF32, NW>(d[i], next);
        }

        uint32_t dead = 0;
        uint32_t lidsel[kQ2];  // bit e: site e's value of direction i bounced off the lid
#pragma unroll
        for (int i = 0; i < kQ2; ++i) lidsel[i] = 0;
        if constexpr (kSolids) {
            if (dirty) {
#pragma unroll
                for (int e = 0; e < V; ++e) dead |= (m[e] >> 31) << e;
#pragma unroll
                for (int i = 1; i < kQ2; ++i) {
#pragma unroll
                    for (int e = 0; e < V; ++e) {
                        if ((m[e] >> i) & 1u) d[i].w[e] = ownv[i].w[e];
                        lidsel[i] |= ((m[e] >> (8 + i)) & 1u) << e;
                    }
                }
            }
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
            float g[kQ2];
#pragma unroll
            for (int i = 0; i < kQ2; ++i) {
                g[i] = K::dec(d[i].w[e]);
                if constexpr (kSolids)
                    if ((lidsel[i] >> e) & 1u) g[i] += a.lidc[i];
            }
            float m0, m1, m2;
            collide2(g, a, m0, m1, m2);
            const bool live = !((dead >> e) & 1u);
#pragma unroll
            for (int i = 0; i < kQ2; ++i) d[i].w[e] = live ? K::enc(g[i]) : 0u;
        }
        if (active) {
            if (dead != (1u << V) - 1u) {
                const StoreBase sb = store_base(dst, own, 4);
#pragma unroll
                for (int i = 0; i < kQ2; ++i) stv_pop<NW>(sb, (uint32_t)i * a.lay.seg * 4u, d[i]);
            }
            // totals of the stored values (dead sites hold zero), in FP64
            double t[kQ2];
#pragma unroll
            for (int i = 0; i < kQ2; ++i) {
                double v = (double)K::dec(d[i].w[0]);
#pragma unroll
                for (int e = 1; e < V; ++e) v += (double)K::dec(d[i].w[e]);
                t[i] = v;
            }
            acc[0] += t[0] + ((t[1] + t[2]) + (t[3] + t[4])) + ((t[5] + t[6]) + (t[7] + t[8]));
            acc[1] += (t[1] - t[2]) + (t[5] + t[6]) - (t[7] + t[8]);
            acc[2] += (t[3] - t[4]) + (t[5] - t[6]) + (t[7] - t[8]);
        }
    }
    store_block_totals(acc, a.partials + 4 * (size_t)blockIdx.x);
    if (a.prev.partials != nullptr && blockIdx.x == 0) append_step_totals(a.prev);
}

// bit i (1..8): site x - c_i is solid; bit 8 + i: it is the lid; bit 31: the site is solid.
__global__ __launch_bounds__(kBlock) void build_masks2d(const uint8_t *flags, int nx, int ny, uint32_t *nbmask)
{
    const int64_t n = (int64_t)nx * ny;
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n; s += (int64_t)gridDim.x * kBlock) {
        const int x = (int)(s % nx), y = (int)(s / nx);
        uint32_t m = flags[s] ? (1u << 31) : 0u;
#pragma unroll
        for (int i = 1; i < kQ2; ++i) {
            int xs = x - CX2[i], ys = y - CY2[i];
            xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
            ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
            const uint8_t f = flags[(int64_t)ys * nx + xs];
            if (f) m |= 1u << i;
            if (f == 2) m |= 1u << (8 + i);
        }
        nbmask[s] = m;
    }
}

// g_i = f_i^eq(rho, u) - w_i in FP64, rounded once (D2Q9 weights).
__global__ __launch_bounds__(kBlock) void init2d(float *dst, Layout lay, int nx, int ny, const double *rho,
                                                 const double *u, const uint8_t *flags)
{
    const int64_t n = (int64_t)nx * ny;
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n; s += (int64_t)gridDim.x * kBlock) {
        const bool solid = flags && flags[s];
        const double r = rho ? rho[s] : 1.0;
        const double ux = u ? u[s] : 0.0, uy = u ? u[n + s] : 0.0;
        const double uu = ux * ux + uy * uy;
        const uint32_t y = (uint32_t)(s / nx), x = (uint32_t)(s - (int64_t)y * nx);
        const uint64_t own = lay.row_base(y) + x;
#pragma unroll
        for (int i = 0; i < kQ2; ++i) {
            const double w = i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
            const double cu = CX2[i] * ux + CY2[i] * uy;
            dst[own + i * lay.seg] = solid ? 0.0f : (float)(w * ((r - 1.0) + r * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu)));
        }
    }
}

__global__ __launch_bounds__(kBlock) void macros2d(const float *src, Layout lay, int nx, int ny, const uint8_t *flags,
                                                   float *rho, float *u)
{
    const int64_t n = (int64_t)nx * ny;
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n; s += (int64_t)gridDim.x * kBlock) {
        float r = 0.0f, ux = 0.0f, uy = 0.0f;
        if (!(flags && flags[s])) {
            const uint32_t y = (uint32_t)(s / nx), x = (uint32_t)(s - (int64_t)y * nx);
            const uint64_t own = lay.row_base(y) + x;
            float g[kQ2];
#pragma unroll
            for (int i = 0; i < kQ2; ++i) g[i] = src[own + i * lay.seg];
            const float m = g[0] + ((g[1] + g[2]) + (g[3] + g[4])) + ((g[5] + g[6]) + (g[7] + g[8]));
            const float px = (g[1] - g[2]) + (g[5] + g[6]) - (g[7] + g[8]);
            const float py = (g[3] - g[4]) + (g[5] - g[6]) + (g[7] - g[8]);
            r = 1.0f + m;
            ux = px / r;
            uy = py / r;
        }
        if (rho) rho[s] = r;
        if (u) {
            u[s] = ux;
            u[n + s] = uy;
        }
    }
}

// One byte per 64 consecutive sites: 1 if any of them has a mask bit set.
__global__ __launch_bounds__(kBlock) void build_chunkdirty(const uint32_t *nbmask, int64_t n, uint8_t *dirty)
{
    const int64_t nchunks = (n + 63) / 64;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nchunks; c += (int64_t)gridDim.x * kBlock) {
        const int64_t end = (c + 1) * 64 < n ? (c + 1) * 64 : n;
        uint32_t any = 0;
        for (int64_t s = c * 64; s < end; ++s) any |= nbmask[s];
        dirty[c] = any ? 1 : 0;
    }
}

}  // namespace

hipError_t launch_step2d(int variant, bool solids, const Step2Args &a, int grid, hipStream_t s)
{
    void *fn;
    if (variant == 1)
        fn = solids ? reinterpret_cast<void *>(&step2d<4, true>) : reinterpret_cast<void *>(&step2d<4, false>);
    else if (variant == 2)
        fn = solids ? reinterpret_cast<void *>(&step2d<2, true>) : reinterpret_cast<void *>(&step2d<2, false>);
    else
        fn = solids ? reinterpret_cast<void *>(&step2d<1, true>) : reinterpret_cast<void *>(&step2d<1, false>);
    Step2Args arg = a;
    void *params[] = {&arg};
    return hipLaunchKernel(fn, dim3(grid), dim3(kBlock), params, 0, s);
}

hipError_t launch_masks2d(const uint8_t *flags, int nx, int ny, uint32_t *nbmask, uint8_t *chunkdirty, hipStream_t s)
{
    const int64_t n = (int64_t)nx * ny;
    build_masks2d<<<grid_for((uint64_t)n), kBlock, 0, s>>>(flags, nx, ny, nbmask);
    build_chunkdirty<<<grid_for((uint64_t)(n + 63) / 64), kBlock, 0, s>>>(nbmask, n, chunkdirty);
    return hipGetLastError();
}

hipError_t launch_init2d(void *dst, const Layout &lay, int nx, int ny, const double *rho, const double *u,
                         const uint8_t *flags, hipStream_t s)
{
    init2d<<<grid_for((uint64_t)nx * ny), kBlock, 0, s>>>(static_cast<float *>(dst), lay, nx, ny, rho, u, flags);
    return hipGetLastError();
}

hipError_t launch_macros2d(const void *src, const Layout &lay, int nx, int ny, const uint8_t *flags, float *rho,
                           float *u, hipStream_t s)
{
    macros2d<<<grid_for((uint64_t)nx * ny), kBlock, 0, s>>>(static_cast<const float *>(src), lay, nx, ny, flags, rho,
                                                            u);
    return hipGetLastError();
}

namespace {
__global__ __launch_bounds__(kBlock) void repack2d_kernel(float *planes, float *state, Layout lay, int64_t n,
                                                          int to_state)
{
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < (int64_t)kQ2 * n; k += (int64_t)gridDim.x * kBlock) {
        const int i = (int)(k / n);
        const int64_t s = k - (int64_t)i * n;
        const uint32_t row = (uint32_t)(s / lay.nx);
        const uint64_t li = lay.row_base(row) + (uint64_t)i * lay.seg + (uint64_t)(s - (int64_t)row * lay.nx);
        if (to_state)
            state[li] = planes[k];
        else
            planes[k] = state[li];
    }
}
}  // namespace

hipError_t launch_repack2d(void *planes, void *state, const Layout &lay, int64_t n, bool to_state, hipStream_t s)
{
    repack2d_kernel<<<grid_for((uint64_t)kQ2 * n), kBlock, 0, s>>>(static_cast<float *>(planes),
                                                                   static_cast<float *>(state), lay, n, to_state ? 1 : 0);
    return hipGetLastError();
}

}  // namespace lbm
