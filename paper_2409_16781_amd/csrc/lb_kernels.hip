// D3Q19 BGK fused stream-and-collide kernels for gfx950 (CDNA4).
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
// The update is bound by HBM bandwidth (Section 5.3 finds the paper's kernel
// memory-bound on every device), so the kernels are built around the memory
// stream: 8- or 16-byte loads and stores per lane and population, lanes along
// x, the +-1 x-shift of the pulled rows exchanged between neighbouring lanes
// with one DPP move, one workgroup per tile of 256 lanes, no matrix cores.
#include "lb_internal.h"

namespace lbm {
namespace {

// ---------------------------------------------------------------- lattice --

constexpr int CX[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0};
constexpr int CY[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1};
constexpr int CZ[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
constexpr int OPP[kQ] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
constexpr float W1 = 1.0f / 18.0f, W2 = 1.0f / 36.0f;

__host__ __device__ constexpr int weight_class(int i) { return i == 0 ? 0 : (i < 7 ? 1 : 2); }

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// NW consecutive dwords of one population held by one lane.
template <int NW>
struct Lane {
    uint32_t w[NW];
};

// Populations are read and written once per step: non-temporal accesses by
// default (no reuse to keep in the caches).
#ifndef LB_NT_LOAD
#define LB_NT_LOAD 1
#endif
#ifndef LB_NT_STORE
#define LB_NT_STORE 1
#endif

template <typename T>
__device__ __forceinline__ T ldg(const T *p)
{
#if LB_NT_LOAD
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

template <typename T>
__device__ __forceinline__ void stg(T *p, T v)
{
#if LB_NT_STORE
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

template <int NW>
__device__ __forceinline__ Lane<NW> ldv(const char *p)
{
    Lane<NW> r;
    if constexpr (NW == 4) {
        const u32x4 v = ldg(reinterpret_cast<const u32x4 *>(p));
        r.w[0] = v[0];
        r.w[1] = v[1];
        r.w[2] = v[2];
        r.w[3] = v[3];
    } else if constexpr (NW == 2) {
        const u32x2 v = ldg(reinterpret_cast<const u32x2 *>(p));
        r.w[0] = v[0];
        r.w[1] = v[1];
    } else {
        r.w[0] = ldg(reinterpret_cast<const uint32_t *>(p));
    }
    return r;
}

template <int NW>
__device__ __forceinline__ void stv(char *p, const Lane<NW> &d)
{
    if constexpr (NW == 4) {
        u32x4 v;
        v[0] = d.w[0];
        v[1] = d.w[1];
        v[2] = d.w[2];
        v[3] = d.w[3];
        stg(reinterpret_cast<u32x4 *>(p), v);
    } else if constexpr (NW == 2) {
        u32x2 v;
        v[0] = d.w[0];
        v[1] = d.w[1];
        stg(reinterpret_cast<u32x2 *>(p), v);
    } else {
        stg(reinterpret_cast<uint32_t *>(p), d.w[0]);
    }
}

// Stores of the new state.  With LB_STORE_SC1 (the default) a wave writes
// through a buffer descriptor with the device-scope (sc1) and non-temporal
// bits set; a streaming copy of a 10 GB array ran about 2% faster that way
// on MI355X than with non-temporal global stores alone.  The descriptor
// starts at the wave's first active site (the lowest address of the wave:
// sites, and their row bases, increase with the lane), so every byte offset
// is small and non-negative.
#ifndef LB_STORE_SC1
#define LB_STORE_SC1 1
#endif
constexpr int kStoreAux = 2 | 16;  // nt | sc1

struct StoreBase {
    __amdgpu_buffer_rsrc_t rsrc;
    uint64_t first;  // element offset of the descriptor's base
};

template <int NW>
__device__ __forceinline__ void stv_at(char *dst, const StoreBase &sb, uint64_t elem, int bytes, const Lane<NW> &d)
{
#if LB_STORE_SC1
    const int off = (int)((elem - sb.first) * (uint64_t)bytes);
    if constexpr (NW == 4) {
        typedef unsigned int v4u __attribute__((ext_vector_type(4)));
        v4u v = {d.w[0], d.w[1], d.w[2], d.w[3]};
        __builtin_amdgcn_raw_buffer_store_b128(v, sb.rsrc, off, 0, kStoreAux);
    } else if constexpr (NW == 2) {
        typedef unsigned int v2u __attribute__((ext_vector_type(2)));
        v2u v = {d.w[0], d.w[1]};
        __builtin_amdgcn_raw_buffer_store_b64(v, sb.rsrc, off, 0, kStoreAux);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(d.w[0], sb.rsrc, off, 0, kStoreAux);
    }
#else
    stv<NW>(dst + elem * (uint64_t)bytes, d);
#endif
}

// Descriptor for the stores of the active lanes of a wave (call with every
// lane that will store active).
__device__ __forceinline__ StoreBase store_base(char *dst, uint64_t own, int bytes)
{
    StoreBase sb;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)own);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(own >> 32));
    sb.first = ((uint64_t)hi << 32) | lo;
#if LB_STORE_SC1
    sb.rsrc = __builtin_amdgcn_make_buffer_rsrc(dst + sb.first * (uint64_t)bytes, 0, 0x7fffffff, 0x00020000);
#endif
    return sb;
}

__device__ __forceinline__ uint32_t fastdiv(uint32_t n, const FastDiv &f)
{
    uint32_t t = __umulhi(n, f.m);
    return (uint32_t)(((uint64_t)t + n) >> f.l);
}

// ----------------------------------------------------------------- codecs --
// Each codec maps one stored element (its raw bits, zero-extended to 32 bits)
// to float and back.  Encoding rounds to nearest, ties to even.

template <int C>
struct Codec;

template <>
struct Codec<kF32> {
    static constexpr int kBytes = 4;
    __device__ static float dec(uint32_t b) { return __builtin_bit_cast(float, b); }
    __device__ static uint32_t enc(float v) { return __builtin_bit_cast(uint32_t, v); }
    __device__ static uint32_t enc64(double v) { return __builtin_bit_cast(uint32_t, (float)v); }
};

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// 16-bit codecs also work on the two elements of one dword at once: packed
// conversion (one instruction, round to nearest even) and a dot product with
// (1, 1) for the sum of the pair in FP32.
template <>
struct Codec<kF16> {
    static constexpr int kBytes = 2;
    __device__ static float dec(uint32_t b) { return (float)__builtin_bit_cast(_Float16, (uint16_t)b); }
    __device__ static uint32_t enc(float v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
    __device__ static uint32_t enc64(double v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
    __device__ static void dec2(uint32_t w, float &lo, float &hi)
    {
        lo = dec(w & 0xffffu);
        hi = dec(w >> 16);
    }
    __device__ static uint32_t enc2(float lo, float hi)
    {
        f32x2 v = {lo, hi};
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2));
    }
    __device__ static float sum2(uint32_t w, float acc)
    {
        const f16x2 one = {(_Float16)1.0f, (_Float16)1.0f};
        return __builtin_amdgcn_fdot2(__builtin_bit_cast(f16x2, w), one, acc, false);
    }
};

template <>
struct Codec<kBF16> {
    static constexpr int kBytes = 2;
    __device__ static float dec(uint32_t b) { return __builtin_bit_cast(float, b << 16); }
    __device__ static uint32_t enc(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
    // Nearest bfloat16 to a double (one rounding): pick among the neighbours of
    // the float-rounded candidate.
    __device__ static uint32_t enc64(double v)
    {
        uint32_t b = enc((float)v);
        uint32_t best = b;
        double err = fabs((double)dec(b) - v);
        for (int k = -1; k <= 1; k += 2) {
            uint32_t c = (b + k) & 0xffffu;
            double e = fabs((double)dec(c) - v);
            if (e < err || (e == err && (c & 1u) == 0)) {
                best = c;
                err = e;
            }
        }
        return best;
    }
    __device__ static void dec2(uint32_t w, float &lo, float &hi)
    {
        lo = __builtin_bit_cast(float, w << 16);
        hi = __builtin_bit_cast(float, w & 0xffff0000u);
    }
    __device__ static uint32_t enc2(float lo, float hi)
    {
        f32x2 v = {lo, hi};
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
    }
    __device__ static float sum2(uint32_t w, float acc)
    {
        const bf16x2 one = {(__bf16)1.0f, (__bf16)1.0f};
        return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, w), one, acc, false);
    }
};

// Element e of a lane vector, as raw bits.
template <int C, int NW>
__device__ __forceinline__ uint32_t vget(const Lane<NW> &d, int e)
{
    if constexpr (Codec<C>::kBytes == 4) {
        return d.w[e];
    } else {
        return (e & 1) ? (d.w[e >> 1] >> 16) : (d.w[e >> 1] & 0xffffu);
    }
}

template <int C, int NW>
__device__ __forceinline__ void vset(Lane<NW> &d, int e, uint32_t b)
{
    if constexpr (Codec<C>::kBytes == 4) {
        d.w[e] = b;
    } else {
        d.w[e >> 1] = (e & 1) ? ((d.w[e >> 1] & 0xffffu) | (b << 16)) : ((d.w[e >> 1] & 0xffff0000u) | b);
    }
}

// One element at element offset idx of a population array.
template <int C>
__device__ __forceinline__ uint32_t ld_elem(const char *base, uint64_t idx)
{
    if constexpr (Codec<C>::kBytes == 4)
        return *reinterpret_cast<const uint32_t *>(base + idx * 4);
    else
        return *reinterpret_cast<const uint16_t *>(base + idx * 2);
}

template <int C>
__device__ __forceinline__ void st_elem(char *base, uint64_t idx, uint32_t b)
{
    if constexpr (Codec<C>::kBytes == 4)
        *reinterpret_cast<uint32_t *>(base + idx * 4) = b;
    else
        *reinterpret_cast<uint16_t *>(base + idx * 2) = (uint16_t)b;
}

// -------------------------------------------------------------- collision --
// BGK relaxation with Guo forcing on shifted populations g_i = f_i - w_i:
//   rho = 1 + sum g,  j = sum c g + F/2 (= rho u),
//   g_i' = g_i + omega (g_i^eq - g_i) + S_i,
//   g_i^eq = w_i [drho + 3 c_i.j + (9/2)(c_i.j)(c_i.u) - (3/2) j.u],
//   S_i = (1 - omega/2) w_i [3 c_i.F - 3 u.F + 9 (c_i.u)(c_i.F)].
// Directions i and opp(i) form a pair p with sum s_p = g_i + g_opp and
// difference d_p = g_i - g_opp.  The update is applied as increments:
//   s_p' - s_p = omega (s_p^eq - s_p) + (S_i + S_opp)          (even part)
//   d_p' - d_p = -omega n_p + (S_i - S_opp),  n_p = d_p - d_p^eq (odd part)
//   s_p^eq = 2 w_k (drho - 3/2 j.u) + 9 w_k (c.j)(c.u),  d_p^eq = 6 w_k c.j.
//
// FP32 arrangement.  The collision keeps mass and adds exactly F to the
// momentum.  Rounding must not break those identities by a constant factor,
// or the error grows every step (by about 1e-7 of the momentum per step).
// So every quantity that carries mass or momentum is formed from small
// numbers:
//  - the odd non-equilibrium parts n_p of the six diagonal pairs are computed
//    directly, and the three axis pairs take the remainder of
//    sum_p c_p n_p = m - j = -F/2;
//  - the rest population takes the remainder of the mass increments;
//  - each population changes by g' = g + increment, rounded once.
// With this the FP32 result stays at the rounding level of FP32 storage.

// Half increments of one pair (i, j): hs = (s' - s) / 2, hd = (d' - d) / 2,
//   hs = (omega/2) (s^eq - s) + (S_i + S_opp)/2
//      = cu (q c.j + hC) + base - (omega/2) s,   q = (9/2) omega w_k,
//   base = omega w_k (drho - 3/2 j.u) - 3 (1 - omega/2) w_k u.F.
__device__ __forceinline__ void relax_pair(float &gi, float &gj, float s, float n, float cj, float inv, float base,
                                           float q, float hC, float hD, float hom, float &sum_hs)
{
    const float cu = cj * inv;
    const float hs = cu * (q * cj + hC) + base - hom * s;
    const float hd = hD - hom * n;
    gi = gi + (hs + hd);
    gj = gj + (hs - hd);
    sum_hs += hs;
}

// In: g[19] gathered pre-collision values.  Out: g[19] post-collision values,
// rho and u (pre-collision moments, u with the half-force shift).
__device__ __forceinline__ void collide(float (&g)[kQ], const Coll &p, float &rho, float &ux, float &uy, float &uz)
{
    const float s1 = g[1] + g[2], d1 = g[1] - g[2];
    const float s3 = g[3] + g[4], d3 = g[3] - g[4];
    const float s5 = g[5] + g[6], d5 = g[5] - g[6];
    const float s7 = g[7] + g[10], d7 = g[7] - g[10];
    const float s8 = g[8] + g[9], d8 = g[8] - g[9];
    const float s11 = g[11] + g[14], d11 = g[11] - g[14];
    const float s12 = g[12] + g[13], d12 = g[12] - g[13];
    const float s15 = g[15] + g[18], d15 = g[15] - g[18];
    const float s16 = g[16] + g[17], d16 = g[16] - g[17];
    const float drho = g[0] + ((s1 + s3) + (s5 + s7)) + ((s8 + s11) + (s12 + s15)) + s16;
    const float jx = (d1 + d7 + d8 + d11 + d12) + p.hfx;
    const float jy = (d3 + d7 - d8 + d15 + d16) + p.hfy;
    const float jz = (d5 + d11 - d12 + d15 - d16) + p.hfz;
    rho = 1.0f + drho;
    // 1/rho enters only the second-order terms and the reported velocity; the
    // hardware reciprocal (1 ulp) is accurate enough for both
    const float inv = __builtin_amdgcn_rcpf(rho);
    ux = jx * inv;
    uy = jy * inv;
    uz = jz * inv;
    const float ju = jx * ux + jy * uy + jz * uz;  // rho u.u
    const float uF = ux * p.fx + uy * p.fy + uz * p.fz;
    const float t = drho - 1.5f * ju;
    const float base1 = p.ow1 * t - p.g31 * uF, base2 = p.ow2 * t - p.g32 * uF;

    // odd non-equilibrium parts: diagonals directly, axes as the remainder
    const float c7 = jx + jy, c8 = jx - jy, c11 = jx + jz, c12 = jx - jz, c15 = jy + jz, c16 = jy - jz;
    constexpr float kSixth = 1.0f / 6.0f;
    const float n7 = d7 - kSixth * c7, n8 = d8 - kSixth * c8;
    const float n11 = d11 - kSixth * c11, n12 = d12 - kSixth * c12;
    const float n15 = d15 - kSixth * c15, n16 = d16 - kSixth * c16;
    const float n1 = -p.hfx - ((n7 + n8) + (n11 + n12));
    const float n3 = -p.hfy - ((n7 - n8) + (n15 + n16));
    const float n5 = -p.hfz - ((n11 - n12) + (n15 - n16));

    float sum_hs = 0.0f;
    relax_pair(g[1], g[2], s1, n1, jx, inv, base1, p.q1, p.hC[1], p.hD[1], p.hom, sum_hs);
    relax_pair(g[3], g[4], s3, n3, jy, inv, base1, p.q1, p.hC[3], p.hD[3], p.hom, sum_hs);
    relax_pair(g[5], g[6], s5, n5, jz, inv, base1, p.q1, p.hC[5], p.hD[5], p.hom, sum_hs);
    relax_pair(g[7], g[10], s7, n7, c7, inv, base2, p.q2, p.hC[7], p.hD[7], p.hom, sum_hs);
    relax_pair(g[8], g[9], s8, n8, c8, inv, base2, p.q2, p.hC[8], p.hD[8], p.hom, sum_hs);
    relax_pair(g[11], g[14], s11, n11, c11, inv, base2, p.q2, p.hC[11], p.hD[11], p.hom, sum_hs);
    relax_pair(g[12], g[13], s12, n12, c12, inv, base2, p.q2, p.hC[12], p.hD[12], p.hom, sum_hs);
    relax_pair(g[15], g[18], s15, n15, c15, inv, base2, p.q2, p.hC[15], p.hD[15], p.hom, sum_hs);
    relax_pair(g[16], g[17], s16, n16, c16, inv, base2, p.q2, p.hC[16], p.hD[16], p.hom, sum_hs);
    g[0] = g[0] - 2.0f * sum_hs;
}

// Per-direction totals -> {mass deviation, momentum} of a group of sites.
__device__ __forceinline__ void moments_of_totals(const float (&t)[kQ], float &m, float &px, float &py, float &pz)
{
    m = t[0] + ((t[1] + t[2]) + (t[3] + t[4])) + ((t[5] + t[6]) + (t[7] + t[8])) + ((t[9] + t[10]) + (t[11] + t[12])) +
        ((t[13] + t[14]) + (t[15] + t[16])) + (t[17] + t[18]);
    px = (t[1] - t[2]) + (t[7] + t[8]) - (t[9] + t[10]) + (t[11] + t[12]) - (t[13] + t[14]);
    py = (t[3] - t[4]) + (t[7] - t[8]) + (t[9] - t[10]) + (t[15] + t[16]) - (t[17] + t[18]);
    pz = (t[5] - t[6]) + (t[11] - t[12]) + (t[13] - t[14]) + (t[15] - t[16]) + (t[17] - t[18]);
}

// ------------------------------------------------- FP64 totals per launch --
// Each workgroup of a step reduces its threads' FP64 totals (through LDS in a
// fixed tree) and stores them in its slot of the partials; no fence
// or atomic is needed there, because the totals are reduced by a second,
// stream-ordered kernel (reduce_totals).  Every addition happens in a fixed
// order, so the totals are bitwise reproducible.

__device__ __forceinline__ void store_block_totals(const double (&acc)[4], double *out)
{
    __shared__ double red[4][kBlock];
#pragma unroll
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    if (threadIdx.x < 64) {
        double v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = (red[k][threadIdx.x] + red[k][threadIdx.x + 64]) + (red[k][threadIdx.x + 128] + red[k][threadIdx.x + 192]);
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
        }
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) out[k] = v[k];
        }
    }
}

// Sum v[0..count) (4 doubles each) in a fixed tree; the result is valid in thread 0.
__device__ __forceinline__ void block_sum4(const double *v, int count, double (&out)[4], bool coherent)
{
    __shared__ double tot[4][kBlock];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < count; b += kBlock) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            s[k] += coherent ? __hip_atomic_load(&v[4 * b + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : v[4 * b + k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) tot[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int w = kBlock / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int k = 0; k < 4; ++k) tot[k][threadIdx.x] += tot[k][threadIdx.x + w];
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = tot[k][0];
}

// Workgroup g sums partials [g * kRedChunk, (g + 1) * kRedChunk) into
// gpartials[g]; the last workgroup to finish sums the gpartials in order and
// appends {mass, momentum} of the step to the ring.
__global__ __launch_bounds__(kBlock) void reduce_totals(TotalsArgs a)
{
    __shared__ int is_last;
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

// ------------------------------------------------ step: vector-row kernel --
// A lane owns V consecutive sites of one x-row (nx % V == 0) and moves one
// 4-, 8- or 16-byte vector per population in each direction.  Lanes of a wave
// take consecutive vectors.  For c_x = 0 the pulled vector is the aligned one
// of the source row (y - c_y, z - c_z).  For c_x = +1 (-1) the source is
// shifted by one element: the lane loads the aligned vector and takes the
// missing element from the previous (next) lane's vector with one DPP wave
// shift; the lane at a row end or wave edge loads that element directly,
// wrapping periodically in x.

template <int C, int NW>
__device__ __forceinline__ Lane<NW> shift_in_from_left(const Lane<NW> &d, uint32_t prev_elem)
{
    Lane<NW> r;
    if constexpr (Codec<C>::kBytes == 4) {
        r.w[0] = prev_elem;
#pragma unroll
        for (int j = 1; j < NW; ++j) r.w[j] = d.w[j - 1];
    } else {
        r.w[0] = (d.w[0] << 16) | prev_elem;
#pragma unroll
        for (int j = 1; j < NW; ++j) r.w[j] = __builtin_amdgcn_alignbyte(d.w[j], d.w[j - 1], 2);
    }
    return r;
}

template <int C, int NW>
__device__ __forceinline__ Lane<NW> shift_in_from_right(const Lane<NW> &d, uint32_t next_elem)
{
    Lane<NW> r;
    if constexpr (Codec<C>::kBytes == 4) {
#pragma unroll
        for (int j = 0; j < NW - 1; ++j) r.w[j] = d.w[j + 1];
        r.w[NW - 1] = next_elem;
    } else {
#pragma unroll
        for (int j = 0; j < NW - 1; ++j) r.w[j] = __builtin_amdgcn_alignbyte(d.w[j + 1], d.w[j], 2);
        r.w[NW - 1] = (next_elem << 16) | (d.w[NW - 1] >> 16);
    }
    return r;
}

// Directions with c_x = +1 and c_x = -1.
constexpr int kPlusX[5] = {1, 7, 8, 11, 12};
constexpr int kMinusX[5] = {2, 9, 10, 13, 14};

// DPP wave shifts: lane l receives lane l-1 (shr) or lane l+1 (shl).
__device__ __forceinline__ uint32_t wave_shr1(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ uint32_t wave_shl1(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xf, 0xf, false);
}

template <int V>
__device__ __forceinline__ void store_floats(float *p, const float (&v)[V])
{
    if constexpr (V % 4 == 0) {
#pragma unroll
        for (int h = 0; h < V / 4; ++h)
            *reinterpret_cast<float4 *>(p + 4 * h) = make_float4(v[4 * h], v[4 * h + 1], v[4 * h + 2], v[4 * h + 3]);
    } else if constexpr (V == 2) {
        *reinterpret_cast<float2 *>(p) = make_float2(v[0], v[1]);
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) p[e] = v[e];
    }
}

template <int V>
__device__ __forceinline__ void load_masks(const uint32_t *p, uint32_t (&m)[V])
{
    if constexpr (V % 4 == 0) {
#pragma unroll
        for (int h = 0; h < V / 4; ++h) {
            const u32x4 v = *reinterpret_cast<const u32x4 *>(p + 4 * h);
            m[4 * h + 0] = v[0];
            m[4 * h + 1] = v[1];
            m[4 * h + 2] = v[2];
            m[4 * h + 3] = v[3];
        }
    } else if constexpr (V == 2) {
        const u32x2 v = *reinterpret_cast<const u32x2 *>(p);
        m[0] = v[0];
        m[1] = v[1];
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) m[e] = p[e];
    }
}

// Register budget of the vector-row kernels, as waves per SIMD the compiler
// must fit (the unrolled site loop otherwise favours latency over occupancy):
// three for the 16-bit codecs with 4- or 8-byte vectors (fits without
// spills), no constraint otherwise.
template <int C, int NW>
constexpr int vec_waves()
{
#ifdef LB_VEC_WAVES
    return LB_VEC_WAVES;
#else
    return (Codec<C>::kBytes == 2 && NW <= 2) ? 3 : 1;
#endif
}

// Workgroups are dispatched round-robin over the chip's 8 XCDs (workgroup b
// runs on XCD b mod 8).  Order 1 gives each XCD a contiguous range of tiles:
// a bijection of [0, ntiles) that leaves the last ntiles mod 8 tiles in place.
__device__ __forceinline__ int tile_of(int b, int ntiles, int order)
{
    constexpr int kXcds = 8;
    const int q = ntiles / kXcds;
    if (order == 0 || b >= q * kXcds) return b;
    return (b % kXcds) * q + b / kXcds;
}

// LDS of one workgroup for the x-edge exchange: the last (first) dword of
// each row and wave, for the five c_x = +1 (-1) directions.
struct EdgeLds {
    uint32_t row_last[kBlock][5], row_first[kBlock][5];
    uint32_t wave_last[kBlock / 64][5], wave_first[kBlock / 64][5];
};

// Where the lanes of one tile sit: a lane owns V consecutive sites of one
// stored row (row = y + ny z), starting at x0.
struct TileGeom {
    bool active;              // the lane's slot exists (else it repeats the last slot)
    uint32_t s0;              // stored index of the first site (row * pitch + x0)
    uint32_t row, x0, y, z, ym, yp, zm, zp;
    uint64_t own;             // element offset of the first site, population 0
};

template <int V, bool kPadded>
__device__ __forceinline__ TileGeom tile_geom(const StepArgs &a, int tile)
{
    TileGeom g;
    const uint32_t nx = (uint32_t)a.nx, ny = (uint32_t)a.ny, nz = (uint32_t)a.nz;
    const uint32_t pitch = kPadded ? a.lay.pitch : nx;
    const int slot = tile * kBlock + (int)threadIdx.x;
    g.active = slot < a.nslots;
    g.s0 = (uint32_t)(g.active ? slot : a.nslots - 1) * V;
    g.row = fastdiv(g.s0, a.div_pitch);
    g.x0 = g.s0 - g.row * pitch;
    g.z = fastdiv(g.row, a.div_ny);
    g.y = g.row - g.z * ny;
    g.ym = (g.y == 0 ? ny : g.y) - 1;
    g.yp = (g.y + 1 == ny) ? 0 : g.y + 1;
    g.zm = (g.z == 0 ? nz : g.z) - 1;
    g.zp = (g.z + 1 == nz) ? 0 : g.z + 1;
    g.own = a.lay.row_base(g.row) + g.x0;
    return g;
}

// Pull gather of the 19 populations of a tile's sites from the stored array
// src, with periodic wrap and halfway bounce-back: d[i] = src_i(x - c_i), or
// src_opp(i)(x) where x - c_i is solid.  kSwap gathers the transpose used by
// the adjoint instead: d[i] = src_opp(i)(x - c_i), or src_i(x) where x - c_i
// is solid (that is the value of population opp(i) of the transposed
// streaming).  Returns the lane's dead sites (bit e: site e is solid, or
// padding when kPadded).
template <int C, int NW, bool kSolids, bool kPadded, bool kSwap>
__device__ __forceinline__ uint32_t gather(const StepArgs &a, const char *src, const TileGeom &g, Lane<NW> (&d)[kQ],
                                           EdgeLds &lds)
{
    using K = Codec<C>;
    constexpr int V = NW * 4 / K::kBytes;
    const uint32_t nx = (uint32_t)a.nx, ny = (uint32_t)a.ny;
    const int lane = threadIdx.x & 63;
    const uint32_t x0 = g.x0;

    // start (element offset) of the pulled source row of each population
    uint64_t rb[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const uint32_t ys = CY[i] > 0 ? g.ym : (CY[i] < 0 ? g.yp : g.y);
        const uint32_t zs = CZ[i] > 0 ? g.zm : (CZ[i] < 0 ? g.zp : g.z);
        rb[i] = a.lay.row_base(zs * ny + ys) + (uint64_t)(kSwap ? OPP[i] : i) * a.lay.seg;
    }
#pragma unroll
    for (int i = 0; i < kQ; ++i) d[i] = ldv<NW>(src + (rb[i] + x0) * K::kBytes);

    // +-1 shifts along x (all lanes take part in the DPP moves).  The element
    // a lane needs from beyond its wave or across the periodic wrap comes
    // through LDS when the tile holds whole rows (each element is then read
    // from HBM once), else by a direct load.  The lane holding site nx - 1
    // is the row's right edge (with padded rows that site need not be the
    // last of the vector).
    const bool left_edge = (lane == 0) || (x0 == 0);
    const bool row_end = x0 + V >= nx;
    const bool right_edge = (lane == 63) || row_end;
    const int wave = threadIdx.x >> 6;
    const int rit = (int)threadIdx.x >> a.lg_row_lanes;  // row within the tile
    if (a.lds_edges) {
        __syncthreads();  // the previous readers are done
        if (row_end) {
#pragma unroll
            for (int k = 0; k < 5; ++k) lds.row_last[rit][k] = d[kPlusX[k]].w[NW - 1];
        }
        if (x0 == 0) {
#pragma unroll
            for (int k = 0; k < 5; ++k) lds.row_first[rit][k] = d[kMinusX[k]].w[0];
        }
        if (lane == 63) {
#pragma unroll
            for (int k = 0; k < 5; ++k) lds.wave_last[wave][k] = d[kPlusX[k]].w[NW - 1];
        }
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 5; ++k) lds.wave_first[wave][k] = d[kMinusX[k]].w[0];
        }
        __syncthreads();
    }
    const uint32_t xl = (x0 == 0 ? nx : x0) - 1;
    const uint32_t xr = row_end ? 0 : x0 + V;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int i = kPlusX[k];  // c_x = +1: pull from x - 1
        uint32_t prev = wave_shr1(d[i].w[NW - 1]);
        if (left_edge) {
            if (a.lds_edges) {
                prev = x0 == 0 ? lds.row_last[rit][k] : lds.wave_last[wave - 1][k];
            } else {
                prev = ld_elem<C>(src, rb[i] + xl);
                if constexpr (K::kBytes == 2) prev <<= 16;  // as the upper half of a dword
            }
        }
        if constexpr (K::kBytes == 2) prev >>= 16;
        d[i] = shift_in_from_left<C, NW>(d[i], prev);
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int i = kMinusX[k];  // c_x = -1: pull from x + 1
        uint32_t next = wave_shl1(d[i].w[0]);
        if (right_edge) {
            if (a.lds_edges)
                next = row_end ? lds.row_first[rit][k] : lds.wave_first[wave + 1][k];
            else
                next = ld_elem<C>(src, rb[i] + xr);
        }
        if constexpr (K::kBytes == 2) next &= 0xffffu;
        d[i] = shift_in_from_right<C, NW>(d[i], next);
        if constexpr (kPadded) {
            // site nx - 1 inside the vector: it pulls x = 0 of the row
            if (x0 + V > nx) {
#pragma unroll
                for (int e = 0; e < V - 1; ++e)
                    if (x0 + e + 1 == nx) vset<C, NW>(d[i], e, next);
            }
        }
    }

    // halfway bounce-back: where x - c_i is solid, take the site's own value
    uint32_t dead = 0;
    if constexpr (kPadded) {
#pragma unroll
        for (int e = 1; e < V; ++e) dead |= (x0 + e >= nx ? 1u : 0u) << e;
    }
    if constexpr (kSolids) {
        if (a.rowdirty[g.row]) {
            uint32_t m[V];
            load_masks<V>(a.nbmask + g.s0, m);
#pragma unroll
            for (int e = 0; e < V; ++e) dead |= (m[e] >> 31) << e;
#pragma unroll
            for (int i = 1; i < kQ; ++i) {
                uint32_t sel = 0;  // bit e set: element e bounces back
#pragma unroll
                for (int e = 0; e < V; ++e) sel |= ((m[e] >> i) & 1u) << e;
                if (sel) {
                    const Lane<NW> o = ldv<NW>(src + (g.own + (kSwap ? i : OPP[i]) * a.lay.seg) * K::kBytes);
#pragma unroll
                    for (int e = 0; e < V; ++e)
                        if ((sel >> e) & 1u) vset<C, NW>(d[i], e, vget<C, NW>(o, e));
                }
            }
        }
    }
    return dead;
}

// Collision constants of one site whose x-force is fx (the per-site force
// field added to the uniform one); y and z forces stay uniform.
__device__ __forceinline__ Coll coll_at(const Coll &p, float fx)
{
    Coll q = p;
    q.fx = fx;
    q.hfx = 0.5f * fx;
#pragma unroll
    for (int i = 1; i < kQ; ++i) {
        const float cF = (float)CX[i] * fx + (float)CY[i] * p.fy + (float)CZ[i] * p.fz;
        const float g3 = weight_class(i) == 1 ? p.g31 : p.g32;  // 3 (1 - omega/2) w_i
        q.hC[i] = 3.0f * g3 * cF;
        q.hD[i] = g3 * cF;
    }
    return q;
}

// One tile (kBlock lanes, V sites each) of lattice a: gather with periodic
// wrap and bounce-back, collide, store into dst, and add the FP64 totals of
// the tile's fluid sites to acc.  kPadded: rows are stored with pitch > nx
// (a whole number of vectors); the sites x >= nx of a row are held at zero
// like solid sites and take no part in the totals.  kFField: the x-force of
// each site is the uniform one plus a per-site field (a.fx_field).
template <int C, int NW, bool kSolids, bool kMacros, bool kPadded, bool kFField = false>
__device__ __forceinline__ void tile_update(const StepArgs &a, const char *src, char *dst, int tile,
                                            double (&acc)[4], EdgeLds &lds)
{
    using K = Codec<C>;
    constexpr int V = NW * 4 / K::kBytes;  // sites per lane
    static_assert(!(kPadded && kMacros), "same-pass macros are written for unpadded rows");
    static_assert(!kFField || (K::kBytes == 4 && !kPadded), "force fields: FP32 storage, unpadded rows");
    const Coll &cp = a.coll;
    const TileGeom g = tile_geom<V, kPadded>(a, tile);
    Lane<NW> d[kQ];
    const uint32_t dead = gather<C, NW, kSolids, kPadded, false>(a, src, g, d, lds);

    // collide site by site (16-bit codecs: two sites per dword at a time)
    float mr[V], mu[V], mv[V], mw[V];
    if constexpr (K::kBytes == 4) {
        float fxs[V];
        if constexpr (kFField) {
            load_masks<V>(reinterpret_cast<const uint32_t *>(a.fx_field) + g.s0,
                          reinterpret_cast<uint32_t(&)[V]>(fxs));
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
            float gg[kQ];
#pragma unroll
            for (int i = 0; i < kQ; ++i) gg[i] = K::dec(d[i].w[e]);
            if constexpr (kFField) {
                const Coll q = coll_at(cp, cp.fx + fxs[e]);
                collide(gg, q, mr[e], mu[e], mv[e], mw[e]);
            } else {
                collide(gg, cp, mr[e], mu[e], mv[e], mw[e]);
            }
#pragma unroll
            for (int i = 0; i < kQ; ++i) d[i].w[e] = K::enc(gg[i]);
        }
    } else {
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            float g0[kQ], g1[kQ];
#pragma unroll
            for (int i = 0; i < kQ; ++i) K::dec2(d[i].w[j], g0[i], g1[i]);
            collide(g0, cp, mr[2 * j], mu[2 * j], mv[2 * j], mw[2 * j]);
            collide(g1, cp, mr[2 * j + 1], mu[2 * j + 1], mv[2 * j + 1], mw[2 * j + 1]);
#pragma unroll
            for (int i = 0; i < kQ; ++i) d[i].w[j] = K::enc2(g0[i], g1[i]);
        }
    }

    if (g.active) {
        // Solid (and padding) sites hold zero in both arrays: they are
        // written as zero inside a vector with fluid sites (whole-vector
        // stores) and not at all in an all-solid vector.  The zeros add
        // nothing to the totals below.
        if constexpr (kSolids || kPadded) {
            if (dead) {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    if ((dead >> e) & 1u) {
                        mr[e] = mu[e] = mv[e] = mw[e] = 0.0f;
#pragma unroll
                        for (int i = 0; i < kQ; ++i) vset<C, NW>(d[i], e, 0u);
                    }
                }
            }
        }
        if (dead != (1u << V) - 1u) {
            const StoreBase sb = store_base(dst, g.own, K::kBytes);
#pragma unroll
            for (int i = 0; i < kQ; ++i) stv_at<NW>(dst, sb, g.own + i * a.lay.seg, K::kBytes, d[i]);
        }
        if constexpr (kMacros) {
            const size_t n = (size_t)a.nx * a.ny * a.nz;
            store_floats<V>(a.rho_out + g.s0, mr);
            store_floats<V>(a.u_out + g.s0, mu);
            store_floats<V>(a.u_out + n + g.s0, mv);
            store_floats<V>(a.u_out + 2 * n + g.s0, mw);
        }
        // totals of the values as stored (after rounding), fluid sites only
        float tot[kQ];
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            float t = 0.0f;
#pragma unroll
            for (int j = 0; j < NW; ++j) {
                if constexpr (K::kBytes == 4)
                    t += K::dec(d[i].w[j]);
                else
                    t = K::sum2(d[i].w[j], t);
            }
            tot[i] = t;
        }
        float m, px, py, pz;
        moments_of_totals(tot, m, px, py, pz);
        acc[0] += (double)m;
        acc[1] += (double)px;
        acc[2] += (double)py;
        acc[3] += (double)pz;
    }
}

// ------------------------------------------------------------ adjoint --
// Reverse-mode derivative of one step (FP32 storage).  A step maps the
// stored state S_n to S_{n+1} = C(P S_n): P is the pull streaming with
// bounce-back, C the per-site BGK collision with Guo forcing (Eq. 1-3).  For
// an objective J(S_N) the adjoint lam_n = dJ/dS_n obeys lam_n = P^T nu_n with
// nu_n = (dC/df)^T lam_{n+1} at every site, where f = P S_n.  The kernel of
// step n gathers lam_{n+1} = P^T nu_{n+1} (the transposed pull of the
// previous adjoint array; for the last step lam_N is read at the site
// itself), gathers f from S_n, and writes nu_n.  With rho, u the moments of f
// (u with the half-force shift), w_i the weights and F the site's force:
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
    const char *state = reinterpret_cast<const char *>(a.state);
    const char *lam_src = reinterpret_cast<const char *>(a.lam_in);
    char *nu_out = reinterpret_cast<char *>(a.nu_out);
    const int ntiles = (sa.nslots + kBlock - 1) / kBlock;
    for (int b = blockIdx.x; b < ntiles; b += gridDim.x) {
        const TileGeom g = tile_geom<V, false>(sa, b);
        Lane<NW> d[kQ];
        const uint32_t dead = gather<kF32, NW, kSolids, false, false>(sa, state, g, d, lds);
        // moments of the pulled pre-collision populations (shifted storage)
        float rho[V], ux[V], uy[V], uz[V], fx[V];
        float fxf[V];
        if (sa.fx_field)
            load_masks<V>(reinterpret_cast<const uint32_t *>(sa.fx_field) + g.s0, reinterpret_cast<uint32_t(&)[V]>(fxf));
#pragma unroll
        for (int e = 0; e < V; ++e) {
            float gg[kQ];
#pragma unroll
            for (int i = 0; i < kQ; ++i) gg[i] = K::dec(d[i].w[e]);
            float dr = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                dr += gg[i];
                if (CX[i]) jx += CX[i] * gg[i];
                if (CY[i]) jy += CY[i] * gg[i];
                if (CZ[i]) jz += CZ[i] * gg[i];
            }
            fx[e] = cp.fx + (sa.fx_field ? fxf[e] : 0.0f);
            rho[e] = 1.0f + dr;
            const float inv = 1.0f / rho[e];
            ux[e] = (jx + 0.5f * fx[e]) * inv;
            uy[e] = (jy + cp.hfy) * inv;
            uz[e] = (jz + cp.hfz) * inv;
        }
        // adjoint of the next state at this step's sites
        if constexpr (kFirst) {
#pragma unroll
            for (int i = 0; i < kQ; ++i) d[i] = ldv<NW>(lam_src + (g.own + i * sa.lay.seg) * K::kBytes);
        } else {
            (void)gather<kF32, NW, kSolids, false, true>(sa, lam_src, g, d, lds);
        }
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
                for (int i = 0; i < kQ; ++i) stv_at<NW>(nu_out, sb, g.own + i * sa.lay.seg, K::kBytes, d[i]);
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

// Collide the V sites of a lane (FP32 arithmetic, storage codec C); rho and
// u are not kept.
template <int C, int NW>
__device__ __forceinline__ void collide_lane(Lane<NW> (&d)[kQ], const Coll &cp)
{
    using K = Codec<C>;
    float r, ux, uy, uz;
    if constexpr (K::kBytes == 4) {
#pragma unroll
        for (int e = 0; e < NW; ++e) {
            float gg[kQ];
#pragma unroll
            for (int i = 0; i < kQ; ++i) gg[i] = K::dec(d[i].w[e]);
            collide(gg, cp, r, ux, uy, uz);
#pragma unroll
            for (int i = 0; i < kQ; ++i) d[i].w[e] = K::enc(gg[i]);
        }
    } else {
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            float g0[kQ], g1[kQ];
#pragma unroll
            for (int i = 0; i < kQ; ++i) K::dec2(d[i].w[j], g0[i], g1[i]);
            collide(g0, cp, r, ux, uy, uz);
            collide(g1, cp, r, ux, uy, uz);
#pragma unroll
            for (int i = 0; i < kQ; ++i) d[i].w[j] = K::enc2(g0[i], g1[i]);
        }
    }
}

// FP64 totals of a lane's collided values (dead elements already zero).
template <int C, int NW>
__device__ __forceinline__ void add_totals(const Lane<NW> (&d)[kQ], double (&acc)[4])
{
    using K = Codec<C>;
    float tot[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        float t = 0.0f;
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            if constexpr (K::kBytes == 4)
                t += K::dec(d[i].w[j]);
            else
                t = K::sum2(d[i].w[j], t);
        }
        tot[i] = t;
    }
    float m, px, py, pz;
    moments_of_totals(tot, m, px, py, pz);
    acc[0] += (double)m;
    acc[1] += (double)px;
    acc[2] += (double)py;
    acc[3] += (double)pz;
}

// The lane's solid sites (bit e: site e is solid) and their neighbour masks.
template <int V, bool kSolids>
__device__ __forceinline__ uint32_t own_masks(const StepArgs &a, const TileGeom &g, uint32_t (&m)[V])
{
    uint32_t dead = 0;
#pragma unroll
    for (int e = 0; e < V; ++e) m[e] = 0;
    if constexpr (kSolids) {
        if (a.rowdirty[g.row]) {
            load_masks<V>(a.nbmask + g.s0, m);
#pragma unroll
            for (int e = 0; e < V; ++e) dead |= (m[e] >> 31) << e;
        }
    }
    return dead;
}

// Odd -> even: read, collide, write swapped, all at the site itself.
template <int C, int NW, bool kSolids>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(vec_waves<C, NW>()))) void aa_local(StepArgs a)
{
    using K = Codec<C>;
    constexpr int V = NW * 4 / K::kBytes;
    char *F = reinterpret_cast<char *>(a.dst);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int ntiles = (a.nslots + kBlock - 1) / kBlock;
    for (int b = blockIdx.x; b < ntiles; b += gridDim.x) {
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
                    for (int i = 0; i < kQ; ++i) stv_at<NW>(F, sb, g.own + OPP[i] * a.lay.seg, K::kBytes, d[i]);
                } else {
#pragma unroll
                    for (int i = 0; i < kQ; ++i)
#pragma unroll
                        for (int e = 0; e < V; ++e)
                            if (!((dead >> e) & 1u)) st_elem<C>(F, g.own + OPP[i] * a.lay.seg + e, vget<C, NW>(d[i], e));
                }
            }
            add_totals<C, NW>(d, acc);
        }
    }
    store_block_totals(acc, a.partials + 4 * (size_t)blockIdx.x);
}

// Even -> odd: gather (transposed slots), collide, push to the neighbours.
// (The 16-bit codecs keep the three-wave budget of the two-array step: with
// two waves and no spills the kernel measured 10% slower at 512^3.)
template <int C, int NW, bool kSolids>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(vec_waves<C, NW>()))) void aa_pullpush(StepArgs a)
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
    for (int b = blockIdx.x; b < ntiles; b += gridDim.x) {
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
            add_totals<C, NW>(d, acc);
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

// One step of one lattice: one workgroup per tile (or a capped grid looping
// over tiles); each workgroup stores the FP64 totals of its tiles.
template <int C, int NW, bool kSolids, bool kMacros, bool kFField = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(vec_waves<C, NW>()))) void step_vec(StepArgs a)
{
    __shared__ EdgeLds lds;
    const char *src = reinterpret_cast<const char *>(a.src);
    char *dst = reinterpret_cast<char *>(a.dst);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int ntiles = (a.nslots + kBlock - 1) / kBlock;
    for (int b = blockIdx.x; b < ntiles; b += gridDim.x)
        tile_update<C, NW, kSolids, kMacros, false, kFField>(a, src, dst, tile_of(b, ntiles, a.tile_order), acc, lds);
    store_block_totals(acc, a.partials + 4 * (size_t)blockIdx.x);
}

// One step of a batch of lattices: the tiles of all domains in one launch.
// The domain table is read through the constant address space, so the
// per-tile domain parameters (uniform per workgroup) come in with scalar
// loads and live in scalar registers.
// Address space 4 exists only in the device pass (the host pass parses the
// kernel bodies but generates no code for them).
#if defined(__HIP_DEVICE_COMPILE__)
#define LB_CONSTANT_AS __attribute__((address_space(4)))
#else
#define LB_CONSTANT_AS
#endif
typedef LB_CONSTANT_AS const DomDesc ConstDomDesc;
typedef LB_CONSTANT_AS const int ConstInt;

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

// ---------------------------------------------- step: one site per thread --
// General fallback for any nx: each lane gathers its 19 values with its own
// periodic wrap, no lane exchange.

template <int C, bool kSolids, bool kMacros>
__global__ __launch_bounds__(kBlock) void step_site(StepArgs a)
{
    using K = Codec<C>;
    const Coll &cp = a.coll;
    const uint32_t nx = (uint32_t)a.nx, ny = (uint32_t)a.ny, nz = (uint32_t)a.nz;
    const char *src = reinterpret_cast<const char *>(a.src);
    char *dst = reinterpret_cast<char *>(a.dst);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int ntiles = (a.nslots + kBlock - 1) / kBlock;

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
            g[i] = K::dec(b);
        }
        float rho, ux, uy, uz;
        collide(g, cp, rho, ux, uy, uz);
        float tot[kQ];
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const uint32_t b = K::enc(g[i]);
            st_elem<C>(dst, own + i * a.lay.seg, b);
            tot[i] = K::dec(b);
        }
        if constexpr (kMacros) {
            const size_t n = (size_t)nx * ny * nz;
            a.rho_out[s] = rho;
            a.u_out[s] = ux;
            a.u_out[n + s] = uy;
            a.u_out[2 * n + s] = uz;
        }
        float m, px, py, pz;
        moments_of_totals(tot, m, px, py, pz);
        acc[0] += (double)m;
        acc[1] += (double)px;
        acc[2] += (double)py;
        acc[3] += (double)pz;
    }
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
            st_elem<C>(dst, own + (a.swap ? OPP[i] : i) * a.lay.seg, solid ? 0u : K::enc64(geq));
        }
    }
}

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
    for (int b = blockIdx.x; b < ntiles; b += gridDim.x) {
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

        const bool left_edge = (lane == 0) || (x0 == 0);
        const bool row_end = x0 + V >= nx;
        const bool right_edge = (lane == 63) || row_end;
        if (a.lds_edges) {
            __syncthreads();
            if (row_end) {
#pragma unroll
                for (int k = 0; k < 3; ++k) lds.row_last[rit][k] = d[kPlusX2[k]].w[NW - 1];
            }
            if (x0 == 0) {
#pragma unroll
                for (int k = 0; k < 3; ++k) lds.row_first[rit][k] = d[kMinusX2[k]].w[0];
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
        }
        const uint32_t xl = (x0 == 0 ? nx : x0) - 1;
        const uint32_t xr = row_end ? 0 : x0 + V;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int i = kPlusX2[k];
            uint32_t prev = wave_shr1(d[i].w[NW - 1]);
            if (left_edge) prev = a.lds_edges ? (x0 == 0 ? lds.row_last[rit][k] : lds.wave_last[wave - 1][k])
                                              : ld_elem<kF32>(src, rb[i] + xl);
            d[i] = shift_in_from_left<kF32, NW>(d[i], prev);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int i = kMinusX2[k];
            uint32_t next = wave_shl1(d[i].w[0]);
            if (right_edge) next = a.lds_edges ? (row_end ? lds.row_first[rit][k] : lds.wave_first[wave + 1][k])
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
        float tm = 0.0f, tpx = 0.0f, tpy = 0.0f;
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
                for (int i = 0; i < kQ2; ++i) stv_at<NW>(dst, sb, own + i * a.lay.seg, 4, d[i]);
            }
            // totals of the stored values (dead sites hold zero)
            float t[kQ2];
#pragma unroll
            for (int i = 0; i < kQ2; ++i) {
                float v = 0.0f;
#pragma unroll
                for (int e = 0; e < V; ++e) v += K::dec(d[i].w[e]);
                t[i] = v;
            }
            tm = t[0] + ((t[1] + t[2]) + (t[3] + t[4])) + ((t[5] + t[6]) + (t[7] + t[8]));
            tpx = (t[1] - t[2]) + (t[5] + t[6]) - (t[7] + t[8]);
            tpy = (t[3] - t[4]) + (t[5] - t[6]) + (t[7] - t[8]);
            acc[0] += (double)tm;
            acc[1] += (double)tpx;
            acc[2] += (double)tpy;
        }
    }
    store_block_totals(acc, a.partials + 4 * (size_t)blockIdx.x);
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
    using K = Codec<C>;
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
                g[i] = K::dec(a.aa_phase ? aa_fetch<C>(src, a.lay, a.ny, a.nz, a.flags, a.aa_phase, i, x, row)
                                         : ld_elem<C>(src, own + i * a.lay.seg));
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
        if (x < nx) {
            m = flags[row * nx + x] ? (1u << 31) : 0u;
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

inline int grid_for(uint64_t n, int cap = 65536)
{
    uint64_t g = (n + kBlock - 1) / kBlock;
    if (g > (uint64_t)cap) g = cap;
    return g < 1 ? 1 : (int)g;
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

void *pick_step(int codec, int variant, bool solids, bool macros, bool ffield)
{
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
    void *fn = pick_step(codec, variant, solids, macros, a.fx_field != nullptr);
    StepArgs arg = a;
    void *params[] = {&arg};
    return hipLaunchKernel(fn, dim3(grid), dim3(kBlock), params, 0, s);
}

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

hipError_t launch_batch_step(int codec, int variant, const BatchArgs &a, int grid, hipStream_t s)
{
    BatchArgs arg = a;
    void *params[] = {&arg};
    return hipLaunchKernel(pick_batch(codec, variant), dim3(grid), dim3(kBlock), params, 0, s);
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

hipError_t launch_batch_totals(const BatchTotalsArgs &a, hipStream_t s)
{
    reduce_domains<<<a.ndoms, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

int batch_occupancy(int codec, int variant)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pick_batch(codec, variant), kBlock, 0) != hipSuccess) return 1;
    return nb < 1 ? 1 : nb;
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
        default: macros_kernel<kBF16><<<g, kBlock, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

hipError_t launch_masks(const uint8_t *flags, int nx, int ny, int nz, int pitch, uint32_t *nbmask, uint8_t *rowdirty,
                        hipStream_t s)
{
    build_masks<<<grid_for((uint64_t)pitch * ny * nz), kBlock, 0, s>>>(flags, nx, ny, nz, pitch, nbmask);
    build_rowdirty<<<grid_for((uint64_t)ny * nz), kBlock, 0, s>>>(nbmask, pitch, ny * nz, rowdirty);
    return hipGetLastError();
}

hipError_t launch_zero_solid_macros(const uint8_t *flags, int n, float *rho, float *u, hipStream_t s)
{
    zero_solid_macros<<<grid_for((uint64_t)n), kBlock, 0, s>>>(flags, n, rho, u);
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
