// D3Q19 BGK fused stream-and-collide: the single-lattice step kernels,
// their totals reduction, initialisation, macros, masks, raw-state
// repacking and the copy probe (gfx950, CDNA4).
//
// Method: the lattice Boltzmann equation (paper Eq. 1) with the second-order
// equilibrium (Eq. 2-3, sound speed squared 1/3), fused as in Section 3.1:
// every site gathers its populations from the neighbours' stored
// post-collision values (pull streaming), relaxes them, and writes the result
// into the other array.  Added on top of the paper's D2Q9 scheme: the D3Q19
// velocity set, halfway bounce-back at solid sites, periodic faces and Guo's
// body-force source term.
//
// Storage: one unit-stride vector per population (Section 3.1) inside blocks
// of R x-rows (Layout in lb_internal.h).  What is stored is g_i = f_i - w_i
// (populations shifted by their weights) in FP32, FP16 or BF16; all
// arithmetic is FP32 (Section 3.1.1, "Mixed1").  Summing the shifted values
// gives the density deviation rho - 1 and, because sum_i w_i c_i = 0, the
// momentum directly.
//
// The update is bound by HBM bandwidth (Section 5.4 finds the paper's kernel
// memory-bound on every device), so the kernels are built around the memory
// stream: 8- or 16-byte loads and stores per lane and population, lanes along
// x, the +-1 x-shift of the pulled rows exchanged between neighbouring lanes
// with one DPP move, one workgroup per tile of 256 lanes, no matrix cores.
#include "lb_device.h"

namespace lbm {
namespace {

// Sets n words to zero (a kernel rather than a memset, so that a caller may
// capture it into a graph).
__global__ __launch_bounds__(kBlock) void zero_words(unsigned int *p, int n)
{
    const int i = blockIdx.x * kBlock + (int)threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Workgroup g sums partials [g * kRedChunk, (g + 1) * kRedChunk) into
// gpartials[g]; the last workgroup to finish sums the gpartials in order and
// appends {mass, momentum} of the step to the ring.
__global__ __launch_bounds__(kBlock) void reduce_totals(TotalsArgs a)
{
    __shared__ int is_last;
    // kS16: a flagged step has no totals (it is redone)
    if (a.ovf != nullptr && __hip_atomic_load(a.ovf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return;
    const int first = blockIdx.x * kRedChunk;
    const int count = min(kRedChunk, a.nparts - first);
    double gs[4];
    block_sum4(a.partials + 4 * (size_t)first, count, gs, false);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            __hip_atomic_store(&a.gpartials[4 * blockIdx.x + k], gs[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const unsigned int prev = atomicAdd(a.ticket, 1u);
        is_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    double tot[4];
    block_sum4(a.gpartials, gridDim.x, tot, true);
    if (threadIdx.x == 0) {
        const unsigned long long step = __hip_atomic_load(a.step_counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        double *r = a.ring + 4 * (step % kRingCap);
        r[0] = a.n_fluid + tot[0];
        r[1] = tot[1];
        r[2] = tot[2];
        r[3] = tot[3];
        __hip_atomic_store(a.step_counter, step + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(a.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// One step of one lattice: one workgroup per tile (the grid is the tile
// count); each workgroup stores the FP64 totals of its tile.  In a run
// of steps, workgroup 0 also appends the previous step's totals to the ring
// (a.prev), so a run needs one totals kernel at its end instead of one per
// step.
template <int C, int NW, bool kSolids, bool kMacros, bool kFField = false, bool kPullNT = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(vec_waves<C, NW>()))) void step_vec(StepArgs a)
{
    __shared__ EdgeLds lds;
    if (s16_skip<C>(a)) return;
    const char *src = reinterpret_cast<const char *>(a.src);
    char *dst = reinterpret_cast<char *>(a.dst);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int ntiles = (a.nslots + kBlock - 1) / kBlock;
    if ((int)blockIdx.x < ntiles)
        tile_update<C, NW, kSolids, kMacros, false, kFField, kPullNT>(a, src, dst,
                                                                      tile_of(blockIdx.x, ntiles, a.tile_order), acc, lds);
    store_block_totals(acc, a.partials + 4 * (size_t)blockIdx.x);
    if (a.prev.partials != nullptr && blockIdx.x == 0) append_step_totals(a.prev);
}

// ---------------------------------------------- step: one site per thread --
// General fallback for any nx: each lane gathers its 19 values with its own
// periodic wrap, no lane exchange.

template <int C, bool kSolids, bool kMacros>
__global__ __launch_bounds__(kBlock) void step_site(StepArgs a)
{
    if (s16_skip<C>(a)) return;
    const Coll &cp = a.coll;
    const uint32_t nx = (uint32_t)a.nx, ny = (uint32_t)a.ny, nz = (uint32_t)a.nz;
    const char *src = reinterpret_cast<const char *>(a.src);
    char *dst = reinterpret_cast<char *>(a.dst);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int ntiles = (a.nslots + kBlock - 1) / kBlock;
    Range16 rng;  // kS16: range test of the codes

    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int slot = tile * kBlock + (int)threadIdx.x;
        if (slot >= a.nslots) continue;
        const uint32_t s = (uint32_t)slot;
        const uint32_t row = fastdiv(s, a.div_pitch);
        const uint32_t x = s - row * nx;
        const uint32_t z = fastdiv(row, a.div_ny);
        const uint32_t y = row - z * ny;
        uint32_t mask = 0;
        if constexpr (kSolids) {
            if (a.rowdirty[row]) mask = a.nbmask[s];
            if (mask >> 31) continue;  // solid site: not part of the state
        }
        const uint32_t xm = (x == 0 ? nx : x) - 1, xp = (x + 1 == nx) ? 0 : x + 1;
        const uint32_t ym = (y == 0 ? ny : y) - 1, yp = (y + 1 == ny) ? 0 : y + 1;
        const uint32_t zm = (z == 0 ? nz : z) - 1, zp = (z + 1 == nz) ? 0 : z + 1;
        const uint64_t own = a.lay.row_base(row) + x;
        float g[kQ];
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const uint32_t xs = CX[i] > 0 ? xm : (CX[i] < 0 ? xp : x);
            const uint32_t ys = CY[i] > 0 ? ym : (CY[i] < 0 ? yp : y);
            const uint32_t zs = CZ[i] > 0 ? zm : (CZ[i] < 0 ? zp : z);
            uint32_t b;
            if (kSolids && ((mask >> i) & 1u))
                b = ld_elem<C>(src, own + OPP[i] * a.lay.seg);
            else
                b = ld_elem<C>(src, a.lay.row_base(zs * ny + ys) + i * a.lay.seg + xs);
            g[i] = dec_at<C>(b, a.sc, i);
        }
        float rho, ux, uy, uz;
        collide(g, cp, rho, ux, uy, uz);
        double tot[kQ];
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const uint32_t b = enc_at<C>(g[i], a.sc, i, rng);
            st_elem<C>(dst, own + i * a.lay.seg, b);
            tot[i] = dec64_at<C>(b, a.sc, i);
        }
        if constexpr (kMacros) {
            const size_t n = (size_t)nx * ny * nz;
            a.rho_out[s] = rho;
            a.u_out[s] = ux;
            a.u_out[n + s] = uy;
            a.u_out[2 * n + s] = uz;
        }
        double m, px, py, pz;
        moments_of_totals(tot, m, px, py, pz);
        acc[0] += m;
        acc[1] += px;
        acc[2] += py;
        acc[3] += pz;
    }
    if constexpr (C == kS16) s16_flag(a, rng);
    store_block_totals(acc, a.partials + 4 * (size_t)blockIdx.x);
}

// Solid sites get zero macros in the one-site kernel (it skips them).
__global__ __launch_bounds__(kBlock) void zero_solid_macros(const uint8_t *flags, int n, float *rho, float *u)
{
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n; s += (int64_t)gridDim.x * kBlock) {
        if (flags[s]) {
            rho[s] = 0.0f;
            u[s] = 0.0f;
            u[(size_t)n + s] = 0.0f;
            u[2 * (size_t)n + s] = 0.0f;
        }
    }
}

// -------------------------------------------------------- initialisation --
// g_i = f_i^eq(rho, u) - w_i computed in FP64 and rounded once to storage.

template <int C>
__global__ __launch_bounds__(kBlock) void init_eq(InitArgs a)
{
    using K = Codec<C>;
    char *dst = reinterpret_cast<char *>(a.dst);
    const double w[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < a.n; s += (int64_t)gridDim.x * kBlock) {
        const bool solid = a.flags && a.flags[s];
        const double rho = a.rho ? a.rho[s] : 1.0;
        const double ux = a.u ? a.u[s] : 0.0;
        const double uy = a.u ? a.u[(size_t)a.n + s] : 0.0;
        const double uz = a.u ? a.u[2 * (size_t)a.n + s] : 0.0;
        const double drho = rho - 1.0;
        const double uu = ux * ux + uy * uy + uz * uz;
        const uint32_t r = (uint32_t)s / a.lay.nx;
        const uint64_t own = a.lay.row_base(r) + ((uint32_t)s - r * a.lay.nx);
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
            const double geq = w[weight_class(i)] * (drho + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
            uint32_t b;
            if constexpr (C == kS16) {
                // nearest code (ties to even), saturated (the host's scales leave headroom)
                const double q = fmin(fmax(rint(geq * (double)a.sc.em[weight_class(i)]), -32768.0), 32767.0);
                b = (uint32_t)(uint16_t)(int16_t)q;
            } else {
                b = K::enc64(geq);
            }
            st_elem<C>(dst, own + (a.swap ? OPP[i] : i) * a.lay.seg, solid ? 0u : b);
        }
    }
}

// Largest |g_i^eq| / w_i per weight class (rest, axis, diagonal) over the
// fluid sites of the equilibrium that init_eq writes (as float bits into
// out[0..2]; non-negative floats order like their bits).  The scaled 16-bit
// codec sizes its exponents from them.
__global__ __launch_bounds__(kBlock) void eq_absmax(InitArgs a, unsigned int *out)
{
    float m[3] = {0.0f, 0.0f, 0.0f};  // per weight class
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < a.n; s += (int64_t)gridDim.x * kBlock) {
        if (a.flags && a.flags[s]) continue;
        const double rho = a.rho ? a.rho[s] : 1.0;
        const double ux = a.u ? a.u[s] : 0.0;
        const double uy = a.u ? a.u[(size_t)a.n + s] : 0.0;
        const double uz = a.u ? a.u[2 * (size_t)a.n + s] : 0.0;
        const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
            const double r = (rho - 1.0) + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);  // g_i^eq / w_i
            m[weight_class(i)] = fmaxf(m[weight_class(i)], (float)fabs(r));
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        for (int off = 32; off >= 1; off >>= 1) m[c] = fmaxf(m[c], __shfl_xor(m[c], off, 64));
        if ((threadIdx.x & 63) == 0) atomicMax(out + c, __builtin_bit_cast(unsigned int, m[c]));
    }
}

// Widen the scales of a kS16 array in place: the code of population i is
// divided by 2^shift (of its weight class) and rounded to nearest even (exact
// in float: |q| < 2^15).
__global__ __launch_bounds__(kBlock) void s16_rescale(uint16_t *state, Layout lay, uint64_t elems, Shift16 sh)
{
    for (uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x; k < elems; k += (uint64_t)gridDim.x * kBlock) {
        const int i = (int)((k % lay.blk) / lay.seg);
        const int c = i == 0 ? 0 : (i < 7 ? 1 : 2);
        const float q = (float)(int16_t)state[k];
        state[k] = (uint16_t)(int16_t)(int)rintf(q * __builtin_ldexpf(1.0f, -sh.sh[c]));
    }
}

// ---------------------------------------------------------------- macros --
// rho = 1 + sum g,  u = (sum c g - F/2) / rho of the stored state.

// Element S_i(x) of the stored state at site s = (x, row) of an in-place
// array: phase 1 (even) keeps it in slot opp(i) of x; phase 2 (odd) in slot i
// of x + c_i, or in slot opp(i) of x itself when x + c_i is solid.
template <int C>
__device__ __forceinline__ uint32_t aa_fetch(const char *F, const Layout &lay, int ny, int nz, const uint8_t *flags,
                                             int phase, int i, uint32_t x, uint32_t row)
{
    if (phase == 1) return ld_elem<C>(F, lay.row_base(row) + OPP[i] * lay.seg + x);
    const int nx = (int)lay.nx;
    const int y = (int)(row % (uint32_t)ny), z = (int)(row / (uint32_t)ny);
    int xt = (int)x + CX[i], yt = y + CY[i], zt = z + CZ[i];
    xt = xt < 0 ? xt + nx : (xt >= nx ? xt - nx : xt);
    yt = yt < 0 ? yt + ny : (yt >= ny ? yt - ny : yt);
    zt = zt < 0 ? zt + nz : (zt >= nz ? zt - nz : zt);
    const uint32_t rt = (uint32_t)(zt * ny + yt);
    if (flags && flags[(size_t)rt * nx + xt]) return ld_elem<C>(F, lay.row_base(row) + OPP[i] * lay.seg + x);
    return ld_elem<C>(F, lay.row_base(rt) + i * lay.seg + (uint32_t)xt);
}

template <int C>
__global__ __launch_bounds__(kBlock) void macros_kernel(MacroArgs a)
{
    const char *src = reinterpret_cast<const char *>(a.src);
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < a.n; s += (int64_t)gridDim.x * kBlock) {
        float r = 0.0f, ux = 0.0f, uy = 0.0f, uz = 0.0f;
        if (!(a.flags && a.flags[s])) {
            const uint32_t row = (uint32_t)s / a.lay.nx;
            const uint32_t x = (uint32_t)s - row * a.lay.nx;
            const uint64_t own = a.lay.row_base(row) + x;
            float g[kQ];
#pragma unroll
            for (int i = 0; i < kQ; ++i)
                g[i] = dec_at<C>(a.aa_phase ? aa_fetch<C>(src, a.lay, a.ny, a.nz, a.flags, a.aa_phase, i, x, row)
                                            : ld_elem<C>(src, own + i * a.lay.seg),
                                 a.sc, i);
            float m, px, py, pz;
            moments_of_totals(g, m, px, py, pz);
            r = 1.0f + m;
            const float inv = 1.0f / r;
            const float fxs = a.fx + (a.fx_field ? a.fx_field[s] : 0.0f);
            ux = (px - 0.5f * fxs) * inv;
            uy = (py - 0.5f * a.fy) * inv;
            uz = (pz - 0.5f * a.fz) * inv;
        }
        if (a.rho) a.rho[s] = r;
        if (a.u) {
            a.u[s] = ux;
            a.u[(size_t)a.n + s] = uy;
            a.u[2 * (size_t)a.n + s] = uz;
        }
    }
}

// Raw planes <-> in-place array (see aa_fetch).
template <typename T, int C>
__global__ __launch_bounds__(kBlock) void aa_planes_kernel(T *planes, T *state, Layout lay, int ny, int nz,
                                                           const uint8_t *flags, int phase, int to_state)
{
    const int64_t n = (int64_t)lay.nx * ny * nz;
    const int64_t total = (int64_t)kQ * n;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < total; k += (int64_t)gridDim.x * kBlock) {
        const int i = (int)(k / n);
        const int64_t s = k - (int64_t)i * n;
        const uint32_t row = (uint32_t)(s / lay.nx);
        const uint32_t x = (uint32_t)(s - (int64_t)row * lay.nx);
        if (to_state)
            state[lay.row_base(row) + OPP[i] * lay.seg + x] = planes[k];
        else
            planes[k] = (T)aa_fetch<C>(reinterpret_cast<const char *>(state), lay, ny, nz, flags, phase, i, x, row);
    }
}

// ------------------------------------------------------ neighbour masks --
// bit i (1..18): site x - c_i is solid; bit 31: the site itself is solid.
// Masks are stored like the populations' rows, with pitch >= nx (the padding
// sites of a row get mask 0).

__global__ __launch_bounds__(kBlock) void build_masks(const uint8_t *flags, int nx, int ny, int nz, int pitch,
                                                      uint32_t *nbmask)
{
    const int64_t n = (int64_t)pitch * ny * nz;
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n; s += (int64_t)gridDim.x * kBlock) {
        const int x = (int)(s % pitch);
        const int64_t row = s / pitch;
        const int y = (int)(row % ny), z = (int)(row / ny);
        uint32_t m = 0;
        if (x < nx && flags[row * nx + x]) {
            // a solid site takes no values from anywhere: no neighbour bits,
            // so the gathers issue no bounce-back loads for it
            m = 1u << 31;
        } else if (x < nx) {
#pragma unroll
            for (int i = 1; i < kQ; ++i) {
                int xs = x - CX[i], ys = y - CY[i], zs = z - CZ[i];
                xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
                ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
                zs = zs < 0 ? zs + nz : (zs >= nz ? zs - nz : zs);
                if (flags[((int64_t)zs * ny + ys) * nx + xs]) m |= 1u << i;
            }
        }
        nbmask[s] = m;
    }
}

__global__ __launch_bounds__(kBlock) void build_rowdirty(const uint32_t *nbmask, int pitch, int nrows, uint8_t *rowdirty)
{
    for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * kBlock) {
        uint32_t any = 0;
        for (int x = 0; x < pitch; ++x) any |= nbmask[(size_t)r * pitch + x];
        rowdirty[r] = any ? 1 : 0;
    }
}

// Exclusive prefix count of the dirty rows: rowcum[r] = dirty rows before row
// r, for r = 0..nrows.  A wave covering rows r0..r1 holds a dead site or a
// bounce-back exactly when rowcum[r1 + 1] != rowcum[r0].  One workgroup;
// each pass covers kRowsPerThread rows per thread.
__global__ __launch_bounds__(kBlock) void build_rowcum(const uint8_t *rowdirty, int64_t nrows, uint32_t *rowcum)
{
    constexpr int kRowsPerThread = 16;
    __shared__ uint32_t scan[kBlock];
    uint32_t carry = 0;
    for (int64_t base = 0; base < nrows; base += (int64_t)kBlock * kRowsPerThread) {
        const int64_t first = base + (int64_t)threadIdx.x * kRowsPerThread;
        uint32_t count = 0;
        for (int k = 0; k < kRowsPerThread; ++k)
            if (first + k < nrows && rowdirty[first + k]) ++count;
        scan[threadIdx.x] = count;
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {
            const uint32_t t = (int)threadIdx.x >= off ? scan[threadIdx.x - off] : 0u;
            __syncthreads();
            scan[threadIdx.x] += t;
            __syncthreads();
        }
        uint32_t run = carry + scan[threadIdx.x] - count;  // dirty rows before `first`
        for (int k = 0; k < kRowsPerThread; ++k) {
            if (first + k < nrows) {
                rowcum[first + k] = run;
                if (rowdirty[first + k]) ++run;
            }
        }
        carry += scan[kBlock - 1];
        __syncthreads();  // scan[] is rewritten by the next pass
    }
    if (threadIdx.x == 0) rowcum[nrows] = carry;
}

// ------------------------------------------------------------- raw state --
// Between raw population planes (19 x N elements, plane i holds population i
// of every site in site order) and the storage layout.

template <typename T>
__global__ __launch_bounds__(kBlock) void repack_kernel(T *planes, T *state, Layout lay, int64_t n, int to_state)
{
    const int64_t total = (int64_t)kQ * n;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < total; k += (int64_t)gridDim.x * kBlock) {
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

// ------------------------------------------------------------ copy probe --
// Each workgroup copies 4 KiB: one coalesced 16-byte non-temporal load per
// lane and a store with the same cache policy as the step's stores (the
// fastest streaming copy measured), giving the attainable bandwidth of a
// pass that reads and writes every byte once.

__global__ __launch_bounds__(kBlock) void copy16(const u32x4 *src, u32x4 *dst, uint64_t n16)
{
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n16) {
        Lane<4> v;
        const u32x4 x = __builtin_nontemporal_load(src + i);
        v.w[0] = x[0];
        v.w[1] = x[1];
        v.w[2] = x[2];
        v.w[3] = x[3];
        const StoreBase sb = store_base(reinterpret_cast<char *>(dst), 4 * i, 4);
        stv_at<4>(reinterpret_cast<char *>(dst), sb, 4 * i, 4, v);
    }
}

template <int C, bool S, bool M>
void *step_fn(int variant)
{
    if (variant == 1) return reinterpret_cast<void *>(&step_vec<C, 4, S, M>);
    if (variant == 2) return reinterpret_cast<void *>(&step_vec<C, 2, S, M>);
    if (variant == 3) return reinterpret_cast<void *>(&step_vec<C, 1, S, M>);
    return reinterpret_cast<void *>(&step_site<C, S, M>);
}

template <bool S, bool M>
void *ffield_fn(int variant)
{
    if (variant == 1) return reinterpret_cast<void *>(&step_vec<kF32, 4, S, M, true>);
    if (variant == 2) return reinterpret_cast<void *>(&step_vec<kF32, 2, S, M, true>);
    return reinterpret_cast<void *>(&step_vec<kF32, 1, S, M, true>);
}

// Plain steps of lattices with solids, pulling with non-temporal loads.
template <int C>
void *pull_nt_fn(int variant)
{
    if (variant == 1) return reinterpret_cast<void *>(&step_vec<C, 4, true, false, false, true>);
    if (variant == 2) return reinterpret_cast<void *>(&step_vec<C, 2, true, false, false, true>);
    return reinterpret_cast<void *>(&step_vec<C, 1, true, false, false, true>);
}

// pull_nt: plain steps with solids on the vector-row kernels pull with
// non-temporal loads (ignored elsewhere)
void *pick_step(int codec, int variant, bool solids, bool macros, bool ffield, bool pull_nt = false)
{
    if (pull_nt && solids && !macros && !ffield && variant != 0) {
        switch (codec) {
            case kF32: return pull_nt_fn<kF32>(variant);
            case kF16: return pull_nt_fn<kF16>(variant);
            case kS16: return pull_nt_fn<kS16>(variant);
            default: return pull_nt_fn<kBF16>(variant);
        }
    }
    if (ffield) {  // FP32 storage, vector-row variants only (checked by the caller)
        if (solids) return macros ? ffield_fn<true, true>(variant) : ffield_fn<true, false>(variant);
        return macros ? ffield_fn<false, true>(variant) : ffield_fn<false, false>(variant);
    }
#define LB_PICK(C)                                                                                 \
    if (solids) return macros ? step_fn<C, true, true>(variant) : step_fn<C, true, false>(variant); \
    return macros ? step_fn<C, false, true>(variant) : step_fn<C, false, false>(variant);
    switch (codec) {
        case kF32: LB_PICK(kF32)
        case kF16: LB_PICK(kF16)
        case kS16: LB_PICK(kS16)
        default: LB_PICK(kBF16)
    }
#undef LB_PICK
}

}  // namespace

Coll make_coll(float omega, float fx, float fy, float fz)
{
    Coll p;
    p.hom = 0.5f * omega;
    p.fx = fx;
    p.fy = fy;
    p.fz = fz;
    p.hfx = 0.5f * fx;
    p.hfy = 0.5f * fy;
    p.hfz = 0.5f * fz;
    const float k = 1.0f - 0.5f * omega;
    p.g31 = 3.0f * k * W1;
    p.g32 = 3.0f * k * W2;
    p.ow1 = omega * W1;
    p.ow2 = omega * W2;
    p.q1 = 4.5f * omega * W1;
    p.q2 = 4.5f * omega * W2;
    for (int i = 0; i < kQ; ++i) {
        const float cF = CX[i] * fx + CY[i] * fy + CZ[i] * fz;
        const float gk = k * (weight_class(i) == 1 ? W1 : W2);
        p.hC[i] = 9.0f * gk * cF;
        p.hD[i] = 3.0f * gk * cF;
    }
    return p;
}

int sites_per_thread(int codec, int variant)
{
    const int nw = variant == 1 ? 4 : (variant == 2 ? 2 : (variant == 3 ? 1 : 0));
    if (nw == 0) return 1;
    return nw * 4 / (codec == kF32 ? 4 : 2);
}

int step_occupancy(int codec, int variant, bool solids, bool macros)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pick_step(codec, variant, solids, macros, false), kBlock, 0) !=
        hipSuccess)
        return 1;
    return nb < 1 ? 1 : nb;
}

hipError_t launch_step(int codec, int variant, bool solids, bool macros, const StepArgs &a, int grid, hipStream_t s)
{
    void *fn = pick_step(codec, variant, solids, macros, a.fx_field != nullptr, a.pull_nt != 0);
    StepArgs arg = a;
    void *params[] = {&arg};
    return hipLaunchKernel(fn, dim3(grid), dim3(kBlock), params, 0, s);
}

hipError_t launch_repack(void *planes, void *state, const Layout &lay, int64_t n, int esize, bool to_state,
                         hipStream_t s)
{
    const int g = grid_for((uint64_t)kQ * n);
    if (esize == 4)
        repack_kernel<uint32_t><<<g, kBlock, 0, s>>>(static_cast<uint32_t *>(planes), static_cast<uint32_t *>(state),
                                                     lay, n, to_state ? 1 : 0);
    else
        repack_kernel<uint16_t><<<g, kBlock, 0, s>>>(static_cast<uint16_t *>(planes), static_cast<uint16_t *>(state),
                                                     lay, n, to_state ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_aa_planes(void *planes, void *state, const Layout &lay, int ny, int nz, const uint8_t *flags,
                            int esize, int phase, bool to_state, hipStream_t s)
{
    const int g = grid_for((uint64_t)kQ * lay.nx * ny * nz);
    if (esize == 4)
        aa_planes_kernel<uint32_t, kF32><<<g, kBlock, 0, s>>>(static_cast<uint32_t *>(planes),
                                                              static_cast<uint32_t *>(state), lay, ny, nz, flags,
                                                              phase, to_state ? 1 : 0);
    else
        aa_planes_kernel<uint16_t, kF16><<<g, kBlock, 0, s>>>(static_cast<uint16_t *>(planes),
                                                              static_cast<uint16_t *>(state), lay, ny, nz, flags,
                                                              phase, to_state ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_totals(const TotalsArgs &a, hipStream_t s)
{
    const int g = (a.nparts + kRedChunk - 1) / kRedChunk;
    reduce_totals<<<g, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_init(int codec, const InitArgs &a, hipStream_t s)
{
    const int g = grid_for((uint64_t)a.n);
    switch (codec) {
        case kF32: init_eq<kF32><<<g, kBlock, 0, s>>>(a); break;
        case kF16: init_eq<kF16><<<g, kBlock, 0, s>>>(a); break;
        case kS16: init_eq<kS16><<<g, kBlock, 0, s>>>(a); break;
        default: init_eq<kBF16><<<g, kBlock, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

hipError_t launch_macros(int codec, const MacroArgs &a, hipStream_t s)
{
    const int g = grid_for((uint64_t)a.n);
    switch (codec) {
        case kF32: macros_kernel<kF32><<<g, kBlock, 0, s>>>(a); break;
        case kF16: macros_kernel<kF16><<<g, kBlock, 0, s>>>(a); break;
        case kS16: macros_kernel<kS16><<<g, kBlock, 0, s>>>(a); break;
        default: macros_kernel<kBF16><<<g, kBlock, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

hipError_t launch_masks(const uint8_t *flags, int nx, int ny, int nz, int pitch, uint32_t *nbmask, uint8_t *rowdirty,
                        uint32_t *rowcum, hipStream_t s)
{
    build_masks<<<grid_for((uint64_t)pitch * ny * nz), kBlock, 0, s>>>(flags, nx, ny, nz, pitch, nbmask);
    build_rowdirty<<<grid_for((uint64_t)ny * nz), kBlock, 0, s>>>(nbmask, pitch, ny * nz, rowdirty);
    build_rowcum<<<1, kBlock, 0, s>>>(rowdirty, (int64_t)ny * nz, rowcum);
    return hipGetLastError();
}

hipError_t launch_zero_solid_macros(const uint8_t *flags, int n, float *rho, float *u, hipStream_t s)
{
    zero_solid_macros<<<grid_for((uint64_t)n), kBlock, 0, s>>>(flags, n, rho, u);
    return hipGetLastError();
}

hipError_t launch_eq_absmax(const InitArgs &a, unsigned int *out, hipStream_t s)
{
    zero_words<<<1, kBlock, 0, s>>>(out, 3);
    eq_absmax<<<grid_for((uint64_t)a.n, 4096), kBlock, 0, s>>>(a, out);
    return hipGetLastError();
}

hipError_t launch_s16_rescale(void *state, const Layout &lay, uint64_t elems, const Shift16 &sh, hipStream_t s)
{
    s16_rescale<<<grid_for(elems), kBlock, 0, s>>>(static_cast<uint16_t *>(state), lay, elems, sh);
    return hipGetLastError();
}

hipError_t launch_zero_words(unsigned int *p, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    zero_words<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, uint64_t bytes, hipStream_t s)
{
    const uint64_t n16 = bytes / 16;
    const uint64_t grid = (n16 + kBlock - 1) / kBlock;
    copy16<<<dim3((unsigned)grid), kBlock, 0, s>>>(reinterpret_cast<const u32x4 *>(src), reinterpret_cast<u32x4 *>(dst),
                                                   n16);
    return hipGetLastError();
}

}  // namespace lbm
