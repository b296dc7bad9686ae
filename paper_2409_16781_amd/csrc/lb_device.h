// Device building blocks shared by the kernel sources (one copy per
// translation unit: everything here is inline or a template in an unnamed
// namespace).
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
#pragma once
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

// kNT = false: an ordinary (cached) load.  Kernels with solid sites pull
// with cached loads by default: a bounce-back load of a site's own opposite
// population then tends to hit the L2 line that the tile pulling that
// population from the site's row has just fetched, instead of fetching a
// whole line for one lane's element again.  Where few sites bounce back
// (walls), non-temporal pulls can be faster; the launch-shape tuner times
// both.
template <typename T, bool kNT = true>
__device__ __forceinline__ T ldg(const T *p)
{
#if LB_NT_LOAD
    if constexpr (kNT) return __builtin_nontemporal_load(p);
#endif
    return *p;
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

template <int NW, bool kNT = true>
__device__ __forceinline__ Lane<NW> ldv(const char *p)
{
    Lane<NW> r;
    if constexpr (NW == 4) {
        const u32x4 v = ldg<u32x4, kNT>(reinterpret_cast<const u32x4 *>(p));
        r.w[0] = v[0];
        r.w[1] = v[1];
        r.w[2] = v[2];
        r.w[3] = v[3];
    } else if constexpr (NW == 2) {
        const u32x2 v = ldg<u32x2, kNT>(reinterpret_cast<const u32x2 *>(p));
        r.w[0] = v[0];
        r.w[1] = v[1];
    } else {
        r.w[0] = ldg<uint32_t, kNT>(reinterpret_cast<const uint32_t *>(p));
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
    uint32_t lane;   // byte offset of the lane's own element from that base
    char *own;       // the lane's own element (stores without the descriptor)
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
    sb.lane = (uint32_t)(own - sb.first) * (uint32_t)bytes;
#if LB_STORE_SC1
    sb.rsrc = __builtin_amdgcn_make_buffer_rsrc(dst + sb.first * (uint64_t)bytes, 0, 0x7fffffff, 0x00020000);
    sb.own = nullptr;
#else
    sb.own = dst + own * (uint64_t)bytes;
#endif
    return sb;
}

// Store of a lane vector at byte offset off (wave-uniform: the population's
// segment in the block) from the lane's own element.  A block holds fewer
// than 2^30 bytes and a wave's sites lie in at most two blocks unless the
// blocks are tiny, so lane + off stays below 2^31.
template <int NW>
__device__ __forceinline__ void stv_pop(const StoreBase &sb, uint32_t off, const Lane<NW> &d)
{
#if LB_STORE_SC1
    const int o = (int)(sb.lane + off);
    if constexpr (NW == 4) {
        typedef unsigned int v4u __attribute__((ext_vector_type(4)));
        v4u v = {d.w[0], d.w[1], d.w[2], d.w[3]};
        __builtin_amdgcn_raw_buffer_store_b128(v, sb.rsrc, o, 0, kStoreAux);
    } else if constexpr (NW == 2) {
        typedef unsigned int v2u __attribute__((ext_vector_type(2)));
        v2u v = {d.w[0], d.w[1]};
        __builtin_amdgcn_raw_buffer_store_b64(v, sb.rsrc, o, 0, kStoreAux);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(d.w[0], sb.rsrc, o, 0, kStoreAux);
    }
#else
    stv<NW>(sb.own + off, d);
#endif
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
// conversion (one instruction, round to nearest even).
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
};

// Scaled 16-bit fixed point (see Scale16): the stored word is the int16 q,
// g_i = q 2^-e_i.  Decoding puts q + 2^15 into the low mantissa bits of the
// float 2^23 (exact), then one FMA applies the scale; encoding is one FMA
// that lands on the integer grid of [2^23, 2^24) (round to nearest even) and
// keeps the low 16 bits, back in two's complement.  A value whose code falls
// outside [-2^15, 2^15) shows as a float outside [2^23, 2^23 + 2^16), i.e.
// one whose upper 16 bits are not 0x4B00 (NaN and infinities included); the
// step kernels OR those bits together and flag such a step.
template <>
struct Codec<kS16> {
    static constexpr int kBytes = 2;
    static constexpr float kBias = 8421376.0f;  // 2^23 + 2^15
    // word (zero-extended) -> the float 2^23 + 2^15 + q
    __device__ static float biased(uint32_t b) { return __builtin_bit_cast(float, ((b & 0xffffu) ^ 0x8000u) + 0x4B000000u); }
    // float on the integer grid of [2^23, 2^24) -> word
    __device__ static uint32_t word(float f) { return (__builtin_bit_cast(uint32_t, f) ^ 0x8000u) & 0xffffu; }
};

constexpr uint32_t kS16Skipped = 8u;  // flag bit of a step skipped after a flagged one

// Stored bits of population i -> value (the scale matters to kS16 only).
template <int C>
__device__ __forceinline__ float dec_at(uint32_t b, const Scale16 &sc, int i)
{
    if constexpr (C == kS16)
        return fmaf(Codec<kS16>::biased(b), sc.dm[weight_class(i)], sc.da[weight_class(i)]);
    else
        return Codec<C>::dec(b);
}

// Range test of the biased kS16 codes per weight class, accumulated while
// encoding and read once per lane: the OR of (bits XOR 0x4B000000) over the
// class's codes has zero upper bits exactly when every code was in range and
// finite (one 3-input logic op per value).
struct Range16 {
    uint32_t o[3];
    __device__ Range16()
    {
#pragma unroll
        for (int c = 0; c < 3; ++c) o[c] = 0u;
    }
    // bit c: a code of weight class c left [-2^15, 2^15) or was not finite
    __device__ uint32_t out_bits() const
    {
        uint32_t b = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) b |= (o[c] >> 16) ? (1u << c) : 0u;
        return b;
    }
};

// Value of population i -> stored bits (kS16 also widens r to the code).
template <int C>
__device__ __forceinline__ uint32_t enc_at(float v, const Scale16 &sc, int i, Range16 &r)
{
    if constexpr (C == kS16) {
        const int c = weight_class(i);
        const float f = fmaf(v, sc.em[c], Codec<kS16>::kBias);
        r.o[c] |= __builtin_bit_cast(uint32_t, f) ^ 0x4B000000u;
        return Codec<kS16>::word(f);
    } else {
        return Codec<C>::enc(v);
    }
}

// Two values of population i packed in one dword (16-bit codecs).
template <int C>
__device__ __forceinline__ void dec2_at(uint32_t w, const Scale16 &sc, int i, float &a, float &b)
{
    if constexpr (C == kS16) {
        a = dec_at<C>(w & 0xffffu, sc, i);
        b = dec_at<C>(w >> 16, sc, i);
    } else {
        Codec<C>::dec2(w, a, b);
    }
}

template <int C>
__device__ __forceinline__ uint32_t enc2_at(float a, float b, const Scale16 &sc, int i, Range16 &r)
{
    if constexpr (C == kS16)
        return enc_at<C>(a, sc, i, r) | (enc_at<C>(b, sc, i, r) << 16);
    else
        return Codec<C>::enc2(a, b);
}

// Exact FP64 value of stored bits b of population i.
template <int C>
__device__ __forceinline__ double dec64_at(uint32_t b, const Scale16 &sc, int i)
{
    if constexpr (C == kS16)
        return (double)(int16_t)(uint16_t)b * (double)sc.dm[weight_class(i)];
    else
        return (double)Codec<C>::dec(b);
}

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

// Per-direction totals -> {mass deviation, momentum} of a group of sites
// (FP32 for the macroscopic fields, FP64 for the conservation totals).
// Sums and differences of the nine opposite pairs first (18 additions), then
// the mass (9 more) and the three momentum components (4 each).
template <typename T>
__device__ __forceinline__ void moments_of_totals(const T (&t)[kQ], T &m, T &px, T &py, T &pz)
{
    const T s1 = t[1] + t[2], d1 = t[1] - t[2];
    const T s3 = t[3] + t[4], d3 = t[3] - t[4];
    const T s5 = t[5] + t[6], d5 = t[5] - t[6];
    const T s7 = t[7] + t[10], d7 = t[7] - t[10];     // (+1, +1, 0) / (-1, -1, 0)
    const T s8 = t[8] + t[9], d8 = t[8] - t[9];       // (+1, -1, 0) / (-1, +1, 0)
    const T s11 = t[11] + t[14], d11 = t[11] - t[14]; // (+1, 0, +1) / (-1, 0, -1)
    const T s12 = t[12] + t[13], d12 = t[12] - t[13]; // (+1, 0, -1) / (-1, 0, +1)
    const T s15 = t[15] + t[18], d15 = t[15] - t[18]; // (0, +1, +1) / (0, -1, -1)
    const T s16 = t[16] + t[17], d16 = t[16] - t[17]; // (0, +1, -1) / (0, -1, +1)
    m = t[0] + (((s1 + s3) + (s5 + s7)) + ((s8 + s11) + (s12 + s15))) + s16;
    px = ((d1 + d7) + (d8 + d11)) + d12;
    py = ((d3 + d7) - (d8 - d15)) + d16;
    pz = ((d5 + d11) - (d12 - d15)) - d16;
}

// Mass and momentum per weight class (rest, axis, diagonal) of integer
// per-population sums t (exact in integers; the rest class has no momentum).
__device__ __forceinline__ void moments_of_totals_by_class(const int (&t)[kQ], int (&m)[3], int (&px)[3], int (&py)[3],
                                                           int (&pz)[3])
{
    const int d1 = t[1] - t[2], d3 = t[3] - t[4], d5 = t[5] - t[6];
    const int d7 = t[7] - t[10], d8 = t[8] - t[9], d11 = t[11] - t[14];
    const int d12 = t[12] - t[13], d15 = t[15] - t[18], d16 = t[16] - t[17];
    m[0] = t[0];
    m[1] = (t[1] + t[2]) + (t[3] + t[4]) + (t[5] + t[6]);
    m[2] = ((t[7] + t[10]) + (t[8] + t[9])) + ((t[11] + t[14]) + (t[12] + t[13])) + ((t[15] + t[18]) + (t[16] + t[17]));
    px[0] = py[0] = pz[0] = 0;
    px[1] = d1;
    py[1] = d3;
    pz[1] = d5;
    px[2] = (d7 + d8) + (d11 + d12);
    py[2] = (d7 - d8) + (d15 + d16);
    pz[2] = (d11 - d12) + (d15 - d16);
}

// FP64 totals of the values a lane stores: every stored element is converted
// to double and summed per direction, then the directions are combined into
// {mass deviation, momentum}, all in FP64 and in a fixed order (dead
// elements hold zero and add nothing).  The stored values are exact in
// double, so a lane's totals carry only FP64 rounding (~1e-16 relative).
template <int C, int NW>
__device__ __forceinline__ void add_lane_totals(const Lane<NW> (&d)[kQ], double (&acc)[4], const Scale16 &sc)
{
    using K = Codec<C>;
    constexpr int V = NW * 4 / K::kBytes;
    double m, px, py, pz;
    if constexpr (C == kS16) {
        // The codes are integers: the lane's mass and momentum per weight
        // class are exact int32 sums (|sum| < 12 V 2^15), each scaled once by
        // its class's 2^-e (exact in double); only the few class terms are
        // added in FP64.
        int q[kQ];
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            q[i] = (int16_t)(uint16_t)vget<C, NW>(d[i], 0);
#pragma unroll
            for (int e = 1; e < V; ++e) q[i] += (int16_t)(uint16_t)vget<C, NW>(d[i], e);
        }
        int qm[3], qx[3], qy[3], qz[3];
        moments_of_totals_by_class(q, qm, qx, qy, qz);
        const double s0 = (double)sc.dm[0], s1 = (double)sc.dm[1], s2 = (double)sc.dm[2];
        m = ((double)qm[0] * s0 + (double)qm[1] * s1) + (double)qm[2] * s2;
        px = (double)qx[1] * s1 + (double)qx[2] * s2;
        py = (double)qy[1] * s1 + (double)qy[2] * s2;
        pz = (double)qz[1] * s1 + (double)qz[2] * s2;
    } else {
        double t[kQ];
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            t[i] = (double)K::dec(vget<C, NW>(d[i], 0));
#pragma unroll
            for (int e = 1; e < V; ++e) t[i] += (double)K::dec(vget<C, NW>(d[i], e));
        }
        moments_of_totals(t, m, px, py, pz);
    }
    acc[0] += m;
    acc[1] += px;
    acc[2] += py;
    acc[3] += pz;
}

// ------------------------------------------------- FP64 totals per launch --
// Each workgroup of a step reduces its threads' FP64 totals (through LDS in a
// fixed tree) and stores them in its slot of the partials; no fence
// or atomic is needed there, because the totals are reduced by a second,
// stream-ordered kernel (reduce_totals).  Every addition happens in a fixed
// order, so the totals are bitwise reproducible.

__device__ __forceinline__ void store_block_totals(const double (&acc)[4], double *out)
{
    // a butterfly within each wave, then the four wave sums through 128 bytes
    // of LDS (a small footprint keeps more workgroups resident per CU)
    __shared__ double red[kBlock / 64][4];
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = acc[k];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) red[threadIdx.x >> 6][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) out[k] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
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

// block_sum4's sum computed by one wave alone, in exactly the same order
// (bitwise the same result, valid in lane 0): lane l plays the threads l,
// l + 64, l + 128 and l + 192 of the block (each first summing its strided
// values), forms the tree's first two levels in registers, and takes the six
// remaining levels with shuffles from the lane w above (no barriers).
__device__ __forceinline__ void wave_sum4(const double *v, int count, double (&out)[4])
{
    typedef double d2 __attribute__((ext_vector_type(2)));
    const int lane = threadIdx.x & 63;
    double a[4][4];  // [block thread l + 64 q][component]
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k) a[q][k] = 0.0;
    // one pass per 256 partials; the four threads' loads of a pass are
    // independent and issued together (32 bytes each)
    for (int base = 0; base < count; base += kBlock) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int b = base + lane + 64 * q;
            if (b < count) {
                const d2 lo = *reinterpret_cast<const d2 *>(v + 4 * (size_t)b);
                const d2 hi = *reinterpret_cast<const d2 *>(v + 4 * (size_t)b + 2);
                a[q][0] += lo[0];
                a[q][1] += lo[1];
                a[q][2] += hi[0];
                a[q][3] += hi[1];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double x = (a[0][k] + a[2][k]) + (a[1][k] + a[3][k]);
#pragma unroll
        for (int w = 32; w >= 1; w >>= 1) x += __shfl_down(x, w, 64);
        out[k] = x;
    }
}

// The totals of one step from its workgroup partials t.partials, summed by a
// single workgroup in the order of reduce_totals (each chunk of kRedChunk
// partials, then the chunk sums, both in the same fixed trees, so the result
// is bitwise the same) and appended to the ring.  The four waves take
// chunks in turn.  The partials were written by an earlier launch, so no
// fence is needed before reading them.
__device__ __forceinline__ void append_step_totals(const TotalsArgs &t)
{
    const int nchunks = (t.nparts + kRedChunk - 1) / kRedChunk;
    for (int c = (int)threadIdx.x >> 6; c < nchunks; c += kBlock / 64) {
        double gs[4];
        wave_sum4(t.partials + 4 * (size_t)c * kRedChunk, min(kRedChunk, t.nparts - c * kRedChunk), gs);
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                __hip_atomic_store(&t.gpartials[4 * c + k], gs[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();  // every wave's chunk sums are stored
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    double tot[4];
    block_sum4(t.gpartials, nchunks, tot, true);
    if (threadIdx.x == 0) {
        const unsigned long long step = __hip_atomic_load(t.step_counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        double *r = t.ring + 4 * (step % kRingCap);
        r[0] = t.n_fluid + tot[0];
        r[1] = tot[1];
        r[2] = tot[2];
        r[3] = tot[3];
        __hip_atomic_store(t.step_counter, step + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
// three for the 16-bit codecs with 4- or 8-byte vectors and two with 16-byte
// vectors (both fit without spills), no constraint otherwise.
template <int C, int NW>
constexpr int vec_waves()
{
#ifdef LB_VEC_WAVES
    return LB_VEC_WAVES;
#else
    return Codec<C>::kBytes == 2 ? (NW <= 2 ? 3 : 2) : 1;
#endif
}

// Workgroups are dispatched round-robin over the chip's 8 XCDs (workgroup b
// runs on XCD b mod 8).  Order 1 gives each XCD a contiguous range of tiles:
// a bijection of [0, ntiles) that leaves the last ntiles mod 8 tiles in place.
// Order 2 keeps consecutive workgroups on consecutive tiles but rotates each
// block of 64 tiles by the block's index, so that tiles at the same place of
// every block (the wall rows of every plane, when a plane is 64 tiles) do
// not all run on the same XCD.
__device__ __forceinline__ int tile_of(int b, int ntiles, int order)
{
    constexpr int kXcds = 8;
    if (order == 2) {
        constexpr int kRot = 64;
        const int blk = b / kRot, base = blk * kRot;
        const int len = ntiles - base < kRot ? ntiles - base : kRot;
        int t = (b - base) + (len == kRot ? (blk & (kRot - 1)) : blk % len);
        if (t >= len) t -= len;
        return base + t;
    }
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
    uint32_t row0;            // row of the tile's first slot (wave-uniform)
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
    g.row0 = fastdiv((uint32_t)(tile * kBlock) * V, a.div_pitch);
    g.z = fastdiv(g.row, a.div_ny);
    g.y = g.row - g.z * ny;
    g.ym = (g.y == 0 ? ny : g.y) - 1;
    g.yp = (g.y + 1 == ny) ? 0 : g.y + 1;
    g.zm = (g.z == 0 ? nz : g.z) - 1;
    g.zp = (g.z + 1 == nz) ? 0 : g.z + 1;
    g.own = a.lay.row_base(g.row) + g.x0;
    return g;
}

// Address space 4 (read-only, read through the scalar cache) exists only in
// the device pass; the host pass parses the kernel bodies but generates no
// code for them.
#if defined(__HIP_DEVICE_COMPILE__)
#define LB_CONSTANT_AS __attribute__((address_space(4)))
#else
#define LB_CONSTANT_AS
#endif
typedef LB_CONSTANT_AS const uint32_t ConstU32;

// Whether any site of the calling wave is solid or has a solid neighbour
// (wave-uniform).  The lanes' rows are increasing, so the wave covers rows
// r0..r1 of lanes 0 and 63; the answer comes from two scalar loads of the
// dirty-row prefix count, with no vector-memory round trip.  All 64 lanes
// must be active.
__device__ __forceinline__ bool wave_dirty(const StepArgs &a, const TileGeom &g)
{
    const uint32_t r0 = __builtin_amdgcn_readfirstlane(g.row);
    const uint32_t r1 = __builtin_amdgcn_readlane(g.row, 63);
    const ConstU32 *rc = (const ConstU32 *)a.rowcum;
    return rc[r1 + 1] != rc[r0];
}

// Pull gather of the 19 populations of a tile's sites from the stored array
// src, with periodic wrap and halfway bounce-back: d[i] = src_i(x - c_i), or
// src_opp(i)(x) where x - c_i is solid.  kSwap gathers the transpose used by
// the adjoint instead: d[i] = src_opp(i)(x - c_i), or src_i(x) where x - c_i
// is solid (that is the value of population opp(i) of the transposed
// streaming).  Returns the lane's dead sites (bit e: site e is solid, or
// padding when kPadded).  kPullNT: with solids, pull with non-temporal loads
// (without solids the pulls always are).
template <int C, int NW, bool kSolids, bool kPadded, bool kSwap, bool kPullNT = false>
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
    for (int i = 0; i < kQ; ++i) d[i] = ldv<NW, !kSolids || kPullNT>(src + (rb[i] + x0) * K::kBytes);
    // Waves with a dead site or a bounce-back issue their neighbour masks
    // right behind the pulls (one round trip for both); the others read no
    // mask at all.
    bool dirty = false;
    uint32_t m[V];
    if constexpr (kSolids) {
        dirty = wave_dirty(a, g);
        if (dirty) load_masks<V>(a.nbmask + g.s0, m);
    }

    // +-1 shifts along x (all lanes take part in the DPP moves).  The element
    // a lane needs from beyond its wave or across the periodic wrap comes
    // through LDS when the lane that holds it is in the same tile (each
    // element is then read from HBM once); only lanes whose source lies in
    // another tile (a row crossing the tile's first or last slot, the
    // tile's outer wave edges) load it directly, issued here behind the
    // pulls so that the wave waits for one round trip, not two.  The lane
    // holding site nx - 1 is the row's right edge (with padded rows that
    // site need not be the last of the vector).
    const bool left_edge = (lane == 0) || (x0 == 0);
    const bool row_end = x0 + V >= nx;
    const bool right_edge = (lane == 63) || row_end;
    const uint32_t xl = (x0 == 0 ? nx : x0) - 1;
    const uint32_t xr = row_end ? 0 : x0 + V;
    const int wave = threadIdx.x >> 6;
    // the row's last site is (nx - 1) / V slots after its first
    const bool prev_lds = a.lds_edges && (x0 == 0 ? (int)threadIdx.x + (int)((nx - 1) / V) < kBlock : wave > 0);
    const bool next_lds = a.lds_edges && (row_end ? (int)threadIdx.x >= (int)(x0 / V) : wave < kBlock / 64 - 1);
    uint32_t eprev[5], enext[5];
    if (left_edge && !prev_lds) {
#pragma unroll
        for (int k = 0; k < 5; ++k) eprev[k] = ld_elem<C>(src, rb[kPlusX[k]] + xl);
    }
    if (right_edge && !next_lds) {
#pragma unroll
        for (int k = 0; k < 5; ++k) enext[k] = ld_elem<C>(src, rb[kMinusX[k]] + xr);
    }
    const int rit = (int)(g.row - g.row0);  // row within the tile
    if (a.lds_edges) {
        __syncthreads();  // the previous readers are done
        if (row_end) {
            // site nx - 1, as the upper half of a dword for 16-bit codecs
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                uint32_t v = d[kPlusX[k]].w[NW - 1];
                if constexpr (kPadded) {
#pragma unroll
                    for (int e = 0; e < V; ++e)
                        if (x0 + e + 1 == nx) v = vget<C, NW>(d[kPlusX[k]], e) << (K::kBytes == 2 ? 16 : 0);
                }
                lds.row_last[rit][k] = v;
            }
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
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int i = kPlusX[k];  // c_x = +1: pull from x - 1
        uint32_t prev = wave_shr1(d[i].w[NW - 1]);
        if (left_edge) {
            if (prev_lds) {
                prev = x0 == 0 ? lds.row_last[rit][k] : lds.wave_last[wave - 1][k];
            } else {
                prev = eprev[k];
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
            if (next_lds)
                next = row_end ? lds.row_first[rit][k] : lds.wave_first[wave + 1][k];
            else
                next = enext[k];
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
        if (dirty) {
#pragma unroll
            for (int e = 0; e < V; ++e) dead |= (m[e] >> 31) << e;
            // The site's own values replace the pulled ones.  A whole vector
            // (and with FP32 storage a single element) is loaded straight
            // into d[i], so these loads are all in flight together; a
            // 16-bit vector with only some sites bouncing back is loaded
            // whole and merged.
#pragma unroll
            for (int i = 1; i < kQ; ++i) {
                uint32_t sel = 0;  // bit e set: element e bounces back
#pragma unroll
                for (int e = 0; e < V; ++e) sel |= ((m[e] >> i) & 1u) << e;
                const char *op = src + (g.own + (kSwap ? i : OPP[i]) * a.lay.seg) * K::kBytes;
                if (sel == (1u << V) - 1u) {
                    d[i] = ldv<NW>(op);
                } else if (sel) {
                    if constexpr (K::kBytes == 4) {
#pragma unroll
                        for (int e = 0; e < V; ++e)
                            if ((sel >> e) & 1u) d[i].w[e] = *reinterpret_cast<const uint32_t *>(op + 4 * e);
                    } else {
                        const Lane<NW> o = ldv<NW>(op);
#pragma unroll
                        for (int e = 0; e < V; ++e)
                            if ((sel >> e) & 1u) vset<C, NW>(d[i], e, vget<C, NW>(o, e));
                    }
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

// Collide the V sites of a lane in place (loaded vectors in, values to store
// out), with their moments in mr/mu/mv/mw.  kFField: site e's x-force is the
// uniform one plus fxs[e] (FP32 storage).  Every kernel that collides a lane
// goes through here, so equal inputs give equal bits whichever kernel runs.
template <int C, int NW, bool kFField>
__device__ __forceinline__ void collide_sites(Lane<NW> (&d)[kQ], const Coll &cp, const Scale16 &sc, Range16 &rng,
                                              const float (&fxs)[NW * 4 / Codec<C>::kBytes],
                                              float (&mr)[NW * 4 / Codec<C>::kBytes],
                                              float (&mu)[NW * 4 / Codec<C>::kBytes],
                                              float (&mv)[NW * 4 / Codec<C>::kBytes],
                                              float (&mw)[NW * 4 / Codec<C>::kBytes])
{
    using K = Codec<C>;
    constexpr int V = NW * 4 / K::kBytes;
    static_assert(!kFField || K::kBytes == 4, "force fields: FP32 storage");
    if constexpr (K::kBytes == 4) {
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
    } else if constexpr (NW >= 4) {
        // 16-byte vectors of 16-bit values (8 sites per lane): one site at a
        // time, its results written back into its half of each dword, so
        // the registers hold the loaded vectors plus one site.
#pragma unroll
        for (int j = 0; j < NW; ++j) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                float gg[kQ];
#pragma unroll
                for (int i = 0; i < kQ; ++i) gg[i] = dec_at<C>(h ? d[i].w[j] >> 16 : d[i].w[j] & 0xffffu, sc, i);
                collide(gg, cp, mr[2 * j + h], mu[2 * j + h], mv[2 * j + h], mw[2 * j + h]);
#pragma unroll
                for (int i = 0; i < kQ; ++i) {
                    const uint32_t b = enc_at<C>(gg[i], sc, i, rng);
                    d[i].w[j] = h ? ((d[i].w[j] & 0xffffu) | (b << 16)) : ((d[i].w[j] & 0xffff0000u) | b);
                }
                // the packed words as they now stand: the next site decodes
                // from these registers, so no two sites' values are live at once
#pragma unroll
                for (int i = 0; i < kQ; ++i) {
#pragma unroll
                    for (int k = 0; k < NW; ++k) asm volatile("" : "+v"(d[i].w[k]));
                }
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            float g0[kQ], g1[kQ];
#pragma unroll
            for (int i = 0; i < kQ; ++i) dec2_at<C>(d[i].w[j], sc, i, g0[i], g1[i]);
            collide(g0, cp, mr[2 * j], mu[2 * j], mv[2 * j], mw[2 * j]);
            collide(g1, cp, mr[2 * j + 1], mu[2 * j + 1], mv[2 * j + 1], mw[2 * j + 1]);
#pragma unroll
            for (int i = 0; i < kQ; ++i) d[i].w[j] = enc2_at<C>(g0[i], g1[i], sc, i, rng);
        }
    }
}

// kS16: a lane whose codes left their class's range, or were not finite (a
// blown-up site: the fixed point would hide a NaN), flags the step with the
// classes to widen; the step is redone from its intact source array with
// wider ranges.
__device__ __forceinline__ void s16_flag(const StepArgs &a, const Range16 &r)
{
    const uint32_t bits = r.out_bits();
    // one atomic per wave at most, and none once the word holds the bits: a
    // step in which millions of codes overflow must not serialise on them
    uint32_t wbits = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) wbits |= __ballot((bits >> c) & 1u) != 0 ? (1u << c) : 0u;
    const unsigned long long active = __ballot(1);
    if (wbits && (uint32_t)(threadIdx.x & 63) == (uint32_t)__builtin_ctzll(active)) {
        const uint32_t have = __hip_atomic_load(&a.ovf[a.par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((have & wbits) != wbits) __hip_atomic_fetch_or(&a.ovf[a.par], wbits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// One tile (kBlock lanes, V sites each) of lattice a: gather with periodic
// wrap and bounce-back, collide, store into dst, and add the FP64 totals of
// the tile's fluid sites to acc.  kPadded: rows are stored with pitch > nx
// (a whole number of vectors); the sites x >= nx of a row are held at zero
// like solid sites and take no part in the totals.  kFField: the x-force of
// each site is the uniform one plus a per-site field (a.fx_field).  kPullNT:
// as in gather.
template <int C, int NW, bool kSolids, bool kMacros, bool kPadded, bool kFField = false, bool kPullNT = false>
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
    const uint32_t dead = gather<C, NW, kSolids, kPadded, false, kPullNT>(a, src, g, d, lds);

    // collide site by site (16-bit codecs: two sites per dword at a time)
    float mr[V], mu[V], mv[V], mw[V];
    Range16 rng;  // kS16: range test of the codes
    float fxs[V];
    if constexpr (kFField) {
        load_masks<V>(reinterpret_cast<const uint32_t *>(a.fx_field) + g.s0, reinterpret_cast<uint32_t(&)[V]>(fxs));
    }
    collide_sites<C, NW, kFField>(d, cp, a.sc, rng, fxs, mr, mu, mv, mw);

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
        if (dead != (1u << V) - 1u && (!kMacros || dst != nullptr)) {
            const StoreBase sb = store_base(dst, g.own, K::kBytes);
            const uint32_t segb = a.lay.seg * (uint32_t)K::kBytes;
#pragma unroll
            for (int i = 0; i < kQ; ++i) stv_pop<NW>(sb, (uint32_t)i * segb, d[i]);
        }
        if constexpr (kMacros) {
            if (a.mom_rec) {
#pragma unroll
                for (int e = 0; e < V; ++e)
                    *reinterpret_cast<float4 *>(a.rho_out + 4 * (size_t)(g.s0 + e)) = make_float4(mr[e], mu[e], mv[e], mw[e]);
            } else {
                const size_t n = (size_t)a.nx * a.ny * a.nz;
                store_floats<V>(a.rho_out + g.s0, mr);
                store_floats<V>(a.u_out + g.s0, mu);
                store_floats<V>(a.u_out + n + g.s0, mv);
                store_floats<V>(a.u_out + 2 * n + g.s0, mw);
            }
        }
        // totals of the values as stored (after rounding), fluid sites only
        add_lane_totals<C, NW>(d, acc, a.sc);
    }
    if constexpr (C == kS16) s16_flag(a, rng);
}

// kS16 steps start here: a step whose predecessor was flagged (overflowed,
// or skipped itself) marks its own parity as skipped and does nothing, so
// the source array of the first flagged step stays intact.
template <int C>
__device__ __forceinline__ bool s16_skip(const StepArgs &a)
{
    if constexpr (C == kS16) {
        if (__hip_atomic_load(&a.ovf[a.par ^ 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
            // the first workgroups mark the skip; the rest find it marked
            if (threadIdx.x == 0 &&
                !(__hip_atomic_load(&a.ovf[a.par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kS16Skipped))
                __hip_atomic_fetch_or(&a.ovf[a.par], kS16Skipped, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return true;
        }
    }
    return false;
}

inline int grid_for(uint64_t n, int cap = 65536)
{
    uint64_t g = (n + kBlock - 1) / kBlock;
    if (g > (uint64_t)cap) g = cap;
    return g < 1 ? 1 : (int)g;
}

}  // namespace
}  // namespace lbm
