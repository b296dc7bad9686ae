// The adjoint (reverse-mode derivative) of the fused D3Q19 step.
#include "lb_device.h"

namespace lbm {
namespace {

// ------------------------------------------------------------ adjoint --
// Reverse-mode derivative of one step (FP32 storage).  A step maps the
// stored state S_n to S_{n+1} = C(P S_n): P is the pull streaming with
// bounce-back, C the per-site BGK collision with Guo forcing (Eq. 1-3).  For
// an objective J(S_N) the adjoint lam_n = dJ/dS_n obeys lam_n = P^T nu_n with
// nu_n = (dC/df)^T lam_{n+1} at every site, where f = P S_n.  The kernel of
// step n gathers lam_{n+1} = P^T nu_{n+1} (the transposed pull of the
// previous adjoint array; for the last step lam_N is read at the site
// itself) and writes nu_n.  The Jacobian of C at a site depends on f only
// through its moments rho and u (u with the half-force shift), which the
// forward step of step n wrote beside its new state; the kernel reads those
// four floats instead of gathering f again.  With w_i the weights and F the
// site's force:
//   nu_j = (1 - omega) lam_j + A + B.(c_j - u) / rho
//   A    = omega sum_i lam_i w_i (1 + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u)
//   B    = sum_i lam_i w_i c_i [3 omega rho + 9 omega rho c_i.u + 9 (1 - omega/2) c_i.F]
//          - 3 (omega rho u + (1 - omega/2) F) sum_i lam_i w_i
// (A and B are lam contracted with dfeq/drho and with dfeq/du + dS/du), and
// the x-force of the site receives
//   dJ/dF_x += B_x / (2 rho) + (1 - omega/2)(3 sum_i lam_i w_i c_ix
//              - 3 u_x sum_i lam_i w_i + 9 sum_i lam_i w_i (c_i.u) c_ix).
// Solid sites keep nu = 0 and no gradient.

template <int NW, bool kFirst, bool kSolids>
__global__ __launch_bounds__(kBlock) void adjoint_vec(AdjArgs a)
{
    using K = Codec<kF32>;
    constexpr int V = NW;
    __shared__ EdgeLds lds;
    const StepArgs &sa = a.s;
    const Coll &cp = sa.coll;
    const float om = 2.0f * cp.hom;        // omega
    const float k1 = 1.0f - cp.hom;        // 1 - omega/2
    const char *lam_src = reinterpret_cast<const char *>(a.lam_in);
    char *nu_out = reinterpret_cast<char *>(a.nu_out);
    const int ntiles = (sa.nslots + kBlock - 1) / kBlock;
    if (const int b = blockIdx.x; b < ntiles) {  // one workgroup per tile
        const TileGeom g = tile_geom<V, false>(sa, b);
        // the moments of step n's pulled populations, as its forward step
        // computed them (one record per site; zero at solid sites)
        float rho[V], ux[V], uy[V], uz[V], fx[V];
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const float4 m = *reinterpret_cast<const float4 *>(a.mom + 4 * (size_t)(g.s0 + e));
            rho[e] = m.x;
            ux[e] = m.y;
            uy[e] = m.z;
            uz[e] = m.w;
        }
        if (sa.fx_field)
            load_masks<V>(reinterpret_cast<const uint32_t *>(sa.fx_field) + g.s0, reinterpret_cast<uint32_t(&)[V]>(fx));
#pragma unroll
        for (int e = 0; e < V; ++e) fx[e] = cp.fx + (sa.fx_field ? fx[e] : 0.0f);
        // adjoint of the next state at this step's sites
        Lane<NW> d[kQ];
        uint32_t dead = 0;
        if constexpr (kFirst) {
#pragma unroll
            for (int i = 0; i < kQ; ++i) d[i] = ldv<NW>(lam_src + (g.own + i * sa.lay.seg) * K::kBytes);
            if constexpr (kSolids) {
                if (wave_dirty(sa, g)) {
                    uint32_t m[V];
                    load_masks<V>(sa.nbmask + g.s0, m);
#pragma unroll
                    for (int e = 0; e < V; ++e) dead |= (m[e] >> 31) << e;
                }
            }
        } else {
            dead = gather<kF32, NW, kSolids, false, true>(sa, lam_src, g, d, lds);
        }
#pragma unroll
        for (int e = 0; e < V; ++e)
            if ((dead >> e) & 1u) rho[e] = 1.0f;  // solid: no moments; the site's output is zero below
        float gF[V];
#pragma unroll
        for (int e = 0; e < V; ++e) {
            float lam[kQ];
#pragma unroll
            for (int k = 0; k < kQ; ++k) lam[k] = K::dec(kFirst ? d[k].w[e] : d[OPP[k]].w[e]);
            const float r = rho[e], u0 = ux[e], u1 = uy[e], u2 = uz[e];
            const float uu = u0 * u0 + u1 * u1 + u2 * u2;
            const float F0 = fx[e], F1 = cp.fy, F2 = cp.fz;
            const float orr = om * r;
            float Lw = 0.0f, A = 0.0f, B0 = 0.0f, B1 = 0.0f, B2 = 0.0f, G0 = 0.0f, H0 = 0.0f;
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const float w = weight_class(i) == 0 ? 1.0f / 3.0f : (weight_class(i) == 1 ? W1 : W2);
                const float lw = lam[i] * w;
                const float cu = CX[i] * u0 + CY[i] * u1 + CZ[i] * u2;
                const float cF = CX[i] * F0 + CY[i] * F1 + CZ[i] * F2;
                Lw += lw;
                A += lw * (1.0f + 3.0f * cu + 4.5f * cu * cu - 1.5f * uu);
                const float t = lw * (3.0f * orr + 9.0f * orr * cu + 9.0f * k1 * cF);
                if (CX[i]) {
                    B0 += CX[i] * t;
                    G0 += CX[i] * lw;
                    H0 += CX[i] * lw * cu;
                }
                if (CY[i]) B1 += CY[i] * t;
                if (CZ[i]) B2 += CZ[i] * t;
            }
            A *= om;
            B0 -= 3.0f * (orr * u0 + k1 * F0) * Lw;
            B1 -= 3.0f * (orr * u1 + k1 * F1) * Lw;
            B2 -= 3.0f * (orr * u2 + k1 * F2) * Lw;
            const float inv = 1.0f / r;
            gF[e] = 0.5f * B0 * inv + k1 * (3.0f * G0 - 3.0f * u0 * Lw + 9.0f * H0);
            const float base = A - (B0 * u0 + B1 * u1 + B2 * u2) * inv;
#pragma unroll
            for (int j = 0; j < kQ; ++j) {
                const float cB = CX[j] * B0 + CY[j] * B1 + CZ[j] * B2;
                const float nu = (1.0f - om) * lam[j] + base + cB * inv;
                d[j].w[e] = K::enc((dead >> e) & 1u ? 0.0f : nu);
            }
        }
        if (g.active) {
            if (dead != (1u << V) - 1u) {
                const StoreBase sb = store_base(nu_out, g.own, K::kBytes);
#pragma unroll
                for (int i = 0; i < kQ; ++i) stv_pop<NW>(sb, (uint32_t)i * sa.lay.seg * (uint32_t)K::kBytes, d[i]);
                float gr[V];
                load_masks<V>(reinterpret_cast<const uint32_t *>(a.grad) + g.s0, reinterpret_cast<uint32_t(&)[V]>(gr));
#pragma unroll
                for (int e = 0; e < V; ++e)
                    if (!((dead >> e) & 1u)) gr[e] += gF[e];
                store_floats<V>(a.grad + g.s0, gr);
            }
        }
    }
}

// ----------------------------------------------------- outlet mass flux --
// J = sum over the fluid sites of the plane x = nx - 1 of rho u_x.  With the
// moments of Section 2 and the Guo half-force shift, rho u_x of a stored
// post-collision state S is sum_i c_ix S_i - F_x / 2 (collision adds exactly F
// to the momentum); the shift by the weights drops out (sum_i w_i c_ix = 0).
// dJ/dS_i = c_ix at those sites, and J depends on the force directly through
// -F_x / 2.

__device__ __forceinline__ bool outlet_fluid(const OutletArgs &a, uint32_t row, uint64_t &site)
{
    site = (uint64_t)row * a.nx + (uint64_t)(a.nx - 1);
    return !(a.flags && a.flags[site]);
}

// Fixed LDS tree over the workgroup's values (same order on every run).
__device__ __forceinline__ double block_tree_sum(double v, double (&red)[kBlock])
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kBlock / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

// First pass: one row (its site x = nx - 1) per thread; workgroup b writes
// the sum of its rows to part[b].
template <int C>
__global__ __launch_bounds__(kBlock) void outlet_flux_rows(OutletArgs a)
{
    using K = Codec<C>;
    __shared__ double red[kBlock];
    const char *src = reinterpret_cast<const char *>(a.state);
    const uint32_t rows = (uint32_t)a.ny * (uint32_t)a.nz;
    const uint32_t r = blockIdx.x * kBlock + threadIdx.x;
    double acc = 0.0;
    uint64_t site;
    if (r < rows && outlet_fluid(a, r, site)) {
        const uint64_t own = a.lay.row_base(r) + (uint64_t)(a.nx - 1);
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            if (CX[i] == 0) continue;
            const double v = (double)K::dec(ld_elem<C>(src, own + i * a.lay.seg));
            acc = CX[i] > 0 ? acc + v : acc - v;
        }
        acc -= 0.5 * ((double)a.fx + (a.fx_field ? (double)a.fx_field[site] : 0.0));
    }
    const double sum = block_tree_sum(acc, red);
    if (threadIdx.x == 0) a.part[blockIdx.x] = sum;
}

// Second pass (one workgroup): each thread sums its share of the parts in
// order, then the tree; J = the total.
__global__ __launch_bounds__(kBlock) void outlet_flux_total(OutletArgs a, int nparts)
{
    __shared__ double red[kBlock];
    double acc = 0.0;
    for (int k = threadIdx.x; k < nparts; k += kBlock) acc += a.part[k];
    const double sum = block_tree_sum(acc, red);
    if (threadIdx.x == 0) a.J[0] = sum;
}

// dJ/dS_N: c_ix at population i of each outlet fluid site (the rest of the
// array was zeroed by the caller).  One thread per (row, population).
__global__ __launch_bounds__(kBlock) void outlet_seed_kernel(OutletArgs a)
{
    const uint64_t rows = (uint64_t)a.ny * (uint64_t)a.nz;
    for (uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x; t < rows * kQ; t += (uint64_t)gridDim.x * kBlock) {
        const uint32_t r = (uint32_t)(t / kQ);
        const int i = (int)(t - (uint64_t)r * kQ);
        uint64_t site;
        if (CX[i] == 0 || !outlet_fluid(a, r, site)) continue;
        a.seed[a.lay.row_base(r) + (uint64_t)i * a.lay.seg + (uint64_t)(a.nx - 1)] = (float)CX[i];
    }
}

// The direct term dJ/dF_x = -1/2 at each outlet fluid site.
__global__ __launch_bounds__(kBlock) void outlet_direct_kernel(OutletArgs a)
{
    const uint64_t rows = (uint64_t)a.ny * (uint64_t)a.nz;
    for (uint64_t r = (uint64_t)blockIdx.x * kBlock + threadIdx.x; r < rows; r += (uint64_t)gridDim.x * kBlock) {
        uint64_t site;
        if (outlet_fluid(a, (uint32_t)r, site)) a.grad[site] -= 0.5f;
    }
}

}  // namespace

int outlet_parts(int ny, int nz) { return (int)(((uint64_t)ny * (uint64_t)nz + kBlock - 1) / kBlock); }

hipError_t launch_outlet_flux(int codec, const OutletArgs &a, hipStream_t s)
{
    const int parts = outlet_parts(a.ny, a.nz);
    if (codec == kF32) outlet_flux_rows<kF32><<<parts, kBlock, 0, s>>>(a);
    else if (codec == kF16) outlet_flux_rows<kF16><<<parts, kBlock, 0, s>>>(a);
    else outlet_flux_rows<kBF16><<<parts, kBlock, 0, s>>>(a);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    outlet_flux_total<<<1, kBlock, 0, s>>>(a, parts);
    return hipGetLastError();
}

hipError_t launch_outlet_seed(const OutletArgs &a, hipStream_t s)
{
    outlet_seed_kernel<<<grid_for((uint64_t)a.ny * a.nz * kQ), kBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_outlet_direct(const OutletArgs &a, hipStream_t s)
{
    outlet_direct_kernel<<<grid_for((uint64_t)a.ny * a.nz), kBlock, 0, s>>>(a);
    return hipGetLastError();
}

namespace {
template <int NW, bool S>
void *adjoint_fn(bool first)
{
    return first ? reinterpret_cast<void *>(&adjoint_vec<NW, true, S>) : reinterpret_cast<void *>(&adjoint_vec<NW, false, S>);
}
template <bool S>
void *pick_adjoint(int variant, bool first)
{
    if (variant == 1) return adjoint_fn<4, S>(first);
    if (variant == 2) return adjoint_fn<2, S>(first);
    return adjoint_fn<1, S>(first);
}
}  // namespace

hipError_t launch_adjoint(int variant, bool first, const AdjArgs &a, int grid, hipStream_t s)
{
    const bool solids = a.s.nbmask != nullptr;
    void *fn = solids ? pick_adjoint<true>(variant, first) : pick_adjoint<false>(variant, first);
    AdjArgs arg = a;
    void *params[] = {&arg};
    return hipLaunchKernel(fn, dim3(grid), dim3(kBlock), params, 0, s);
}

}  // namespace lbm
