// Internal interface between the host runtime (lb_capi.hip) and the kernels
// (lb_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int kQ = 19;
constexpr int kBlock = 256;        // threads per workgroup of every lattice kernel
constexpr int kRingCap = 4096;     // per-step conservation totals kept on the device

enum Codec : int { kF32 = 0, kF16 = 1, kBF16 = 2, kS16 = 3 };

// Scales of the scaled 16-bit fixed-point codec (kS16): population i is
// stored as the int16 q with g_i = q 2^-e_c, one exponent per weight class c
// (rest, axis, diagonal) for the whole lattice.  dm = 2^-e_c, da = -(2^23 +
// 2^15) 2^-e_c (decode: the float with bits 0x4B000000 + (q + 2^15), times
// dm, plus da: exact); em = 2^e_c (encode: g em + 2^23 + 2^15 rounds to
// nearest even at the integer).
struct Scale16 {
    float dm[3], da[3], em[3];
};

struct Shift16 {
    int sh[3];  // per weight class: codes divided by 2^sh (widening the range)
};

// Division by a runtime constant d >= 1 for numerators n < 2^31:
// q = (umulhi(n, m) + n) >> l with l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1
// (Granlund and Montgomery, "Division by invariant integers using multiplication", 1994).
struct FastDiv {
    uint32_t d, m, l;
};

inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    uint64_t m = (((1ull << l) - d) << 32) / d + 1;
    return FastDiv{d, (uint32_t)m, l};
}

// Storage layout of one population array.  The ny*nz x-rows are grouped in
// blocks of R = 2^lg_r consecutive rows (row r = y + ny z); inside a block each
// population keeps its R rows contiguous, one population after the other:
//   element (i, x, r) at (r >> lg_r) * blk + i * seg + (r & (R - 1)) * pitch + x,
// with seg >= R * pitch and blk = 19 seg.  A row occupies pitch >= nx elements
// (pitch > nx only in batches, where rows are padded to whole vectors).
// R = 1 stores the 19 populations of a row one after the other; R >= ny*nz is
// plain structure of arrays.  Blocks of tens of KiB per population keep the
// 38 streams of a step close together in HBM.  A block holds fewer than 2^30
// bytes (checked when a layout is made), so seg and blk are 32-bit and the
// offset of an element inside its block is a 32-bit product.
struct Layout {
    uint32_t nx;     // sites per row
    uint32_t pitch;  // elements per stored row
    uint32_t lg_r;   // log2(rows per block)
    uint32_t seg;    // elements of one population in one block
    uint32_t blk;    // 19 * seg (9 * seg for D2Q9): elements of one block
    uint32_t pad_;
    __host__ __device__ uint64_t row_base(uint32_t r) const
    {
        return (uint64_t)(r >> lg_r) * blk + (r & ((1u << lg_r) - 1u)) * pitch;
    }
};

// Whether a block of q populations of seg elements of esize bytes stays below
// 2^30 bytes: the store offsets from a wave's first element (inside one block,
// or two when the wave's rows cross a block boundary) then fit in 31 bits.
inline bool block_fits(uint64_t seg, int q, int esize)
{
    return seg * (uint64_t)q * (uint64_t)esize < 0x40000000ull;
}

// Per-launch constants of the collision (computed once on the host, in FP32).
struct Coll {
    float hom;             // omega / 2
    float fx, fy, fz;      // body force
    float hfx, hfy, hfz;   // F / 2
    float g31, g32;        // 3 (1 - omega/2) w_k      (axis, diagonal weight)
    float ow1, ow2;        // omega w_k
    float q1, q2;          // (9/2) omega w_k
    float hC[kQ];          // 9 (1 - omega/2) w_k c_i.F
    float hD[kQ];          // 3 (1 - omega/2) w_k c_i.F
};

Coll make_coll(float omega, float fx, float fy, float fz);

constexpr int kRedChunk = 256;   // step-workgroup partials summed by one reduce workgroup (one per thread)

struct TotalsArgs {
    const double *partials;   // 4 doubles per step workgroup
    int nparts;               // step workgroups
    double *gpartials;        // 4 doubles per reduce workgroup
    unsigned int *ticket;     // arrival counter, 0 between launches
    double *ring;             // kRingCap x 4 doubles
    unsigned long long *step_counter;
    double n_fluid;           // number of fluid sites (exact in a double)
    const unsigned int *ovf;  // kS16: overflow flag of the step whose totals these are (set: no
                              // totals appended), or nullptr
};

// Everything one step launch needs.  Pointers are device pointers.
struct StepArgs {
    const void *src;          // stored state (post-collision of the previous step)
    void *dst;                // new state
    Layout lay;
    int nx, ny, nz;
    int nslots;               // rows * pitch / sites_per_thread
    int lds_edges;            // 1: x-edge elements held by a lane of the same tile pass through LDS
    int lg_row_lanes;         // log2(lanes per x-row) (in-place steps: every tile holds whole rows)
    int tile_order;           // 0: tile = workgroup index; 1: contiguous tile ranges per XCD; 2: blocks
                              // of 64 tiles rotated by their index
    int pull_nt;              // host side: 1 = a plain step with solids runs the kernel that pulls with
                              // non-temporal loads (launch_step picks it)
    FastDiv div_pitch, div_ny;
    Coll coll;
    const uint32_t *nbmask;   // per site: bit 31 = site is solid; a fluid site also has bit i set
                              // where x - c_i is solid (a solid site has bit 31 alone)
    const uint8_t *rowdirty;  // per row (y, z): 1 if any site of the row has a bit set in nbmask
    const uint32_t *rowcum;   // rows + 1 entries: rowcum[r] = dirty rows before row r
    float *rho_out;           // optional macros output (N floats) or nullptr
    float *u_out;             // optional macros output (3N floats) or nullptr
    int mom_rec;              // with macros: 1 = rho_out receives one record (rho, u_x, u_y, u_z) per
                              // site (4N floats, site order) and u_out is unused; then dst may be
                              // nullptr (the step writes its moments only)
    double *partials;         // out: 4 doubles per workgroup
    const float *fx_field;    // optional per-site x-force added to coll.fx (N floats, site order) or nullptr
    TotalsArgs prev;          // prev.partials != nullptr: workgroup 0 also appends the totals of the
                              // step whose partials these are (written by the previous launch) to the ring
    Scale16 sc;               // kS16 only
    unsigned int *ovf;        // kS16 only: two flag words; this step ORs into ovf[par] bit c when a code
    int par;                  // of weight class c leaves its range, and skips (ORing bit 3 into ovf[par])
                              // when ovf[par ^ 1] is set
};

// One lattice of a batch.  The step arguments of domain d are s, with the
// source and destination taken from buf[parity] and buf[parity ^ 1].
struct DomDesc {
    StepArgs s;               // src, dst, rho_out, u_out and partials unused
    void *buf[2];             // the domain's two population arrays
    int tile_begin;           // first tile of the domain in the batch's tile list
    int ntiles;               // tiles of the domain
    double n_fluid;           // fluid sites of the domain
};

// Per-domain totals of one batch step: domain d sums the partials of its
// tiles (in order) into ring[d][step % kRingCap].
struct BatchTotalsArgs {
    const DomDesc *doms;
    int ndoms;
    const double *partials;   // 4 doubles per tile
    unsigned int *ticket;     // arrival counter, 0 between launches
    double *ring;             // ndoms x kRingCap x 4 doubles
    unsigned long long *step_counter;
};

// A step of a batch: every tile of every domain in one launch.
struct BatchArgs {
    const DomDesc *doms;      // device table, one entry per domain
    const int *tile_dom;      // per tile: its domain
    int ntiles;               // tiles of all domains
    int parity;               // source arrays are buf[parity]
    int tile_order;           // as in StepArgs
    double *partials;         // out: 4 doubles per tile
    BatchTotalsArgs prev;     // prev.partials != nullptr: workgroup 0 also appends the previous step's totals
};

// One adjoint step (FP32 storage): see adjoint_vec in lb_adjoint_kernels.hip.
struct AdjArgs {
    StepArgs s;               // geometry, masks, collision constants, force field
    const float *mom;         // moments of step n's pulled populations: one record (rho, u_x, u_y,
                              // u_z) per site, site order, as written by its forward step
    const void *lam_in;       // first step: dJ/dS_N (read at each site); else nu_{n+1}
    void *nu_out;             // nu_n = (dC/df)^T lam_{n+1}
    float *grad;              // N floats (site order): += dJ/dF_x of this step
};

// The outlet mass flux objective: J = sum over the fluid sites of the plane
// x = nx - 1 of rho u_x = sum_i c_ix S_i - F_x / 2 (S the stored state).
struct OutletArgs {
    const void *state;        // stored state, storage layout (two-array storage)
    float *seed;              // storage-layout FP32 array: dJ/dS_N = c_ix at the outlet's fluid sites
    float *grad;              // N floats, site order: the direct term -1/2 at the outlet's fluid sites
    double *J;                // device double receiving J
    double *part;             // outlet_parts(ny, nz) doubles: the per-workgroup sums of J
    Layout lay;
    int nx, ny, nz;
    const uint8_t *flags;     // device flags or nullptr (all fluid)
    float fx;                 // uniform x-force
    const float *fx_field;    // per-site x-force (N floats) or nullptr
};

// One step of a two-dimensional D2Q9 lattice (FP32 storage of f - w).
struct Step2Args {
    const void *src;
    void *dst;
    Layout lay;               // rows are the ny lines of x (one block layout as in 3-D)
    int nx, ny;
    int nslots;               // ny * nx / sites per lane
    int lds_edges, lg_row_lanes;
    FastDiv div_pitch;
    float hom;                // omega / 2
    float ow1, ow2;           // omega w (axis 1/9, diagonal 1/36)
    float q1, q2;             // (9/2) omega w
    float lidc[9];            // 6 w_i (c_i . u_lid): added to a value bounced off the lid
    const uint32_t *nbmask;   // bit i: site x - c_i solid; bit 8 + i: that site is the lid; bit 31: own solid
    const uint8_t *chunkdirty;  // per 64 sites (site s in chunk s / 64): any mask bit set
    double *partials;         // 4 doubles per workgroup (mass, px, py, 0)
    TotalsArgs prev;          // as in StepArgs: the previous step's totals appended by workgroup 0
};

// The reduction of one step's partials into the ring of per-step totals.

struct InitArgs {
    void *dst;
    Layout lay;
    int n;                    // N (sites, x fastest; inputs are unpadded)
    const double *rho;        // N or nullptr
    const double *u;          // 3N or nullptr
    const uint8_t *flags;     // device flags or nullptr
    int swap;                 // 1: population i goes to slot opp(i) (in-place storage, even phase)
    Scale16 sc;               // kS16 only
};

struct MacroArgs {
    const void *src;
    Layout lay;
    int n;
    int ny, nz;
    int aa_phase;             // in-place storage: 1 even (swapped slots), 2 odd (pulled); 0: two arrays
    float fx, fy, fz;
    const float *fx_field;    // per-site x-force added to fx (N floats) or nullptr
    const uint8_t *flags;
    float *rho;
    float *u;
    Scale16 sc;               // kS16 only
};

// Launchers (lb_kernels.hip).  variant: 0 = one site per thread; 1 / 2 / 3 = vector
// rows with 16- / 8- / 4-byte accesses per lane and population plane.
hipError_t launch_step(int codec, int variant, bool solids, bool macros, const StepArgs &a, int grid,
                       hipStream_t s);
hipError_t launch_totals(const TotalsArgs &a, hipStream_t s);
hipError_t launch_init(int codec, const InitArgs &a, hipStream_t s);
hipError_t launch_macros(int codec, const MacroArgs &a, hipStream_t s);
// Neighbour masks of a (nx, ny, nz) lattice stored with row pitch >= nx
// (mask of site (x, row) at row * pitch + x); rowdirty per row and its
// exclusive prefix count rowcum (ny * nz + 1 entries).
hipError_t launch_masks(const uint8_t *flags, int nx, int ny, int nz, int pitch, uint32_t *nbmask, uint8_t *rowdirty,
                        uint32_t *rowcum, hipStream_t s);
hipError_t launch_zero_solid_macros(const uint8_t *flags, int n, float *rho, float *u, hipStream_t s);
hipError_t launch_copy(const void *src, void *dst, uint64_t bytes, hipStream_t s);
hipError_t launch_zero_words(unsigned int *p, int n, hipStream_t s);  // n words set to 0 by a kernel
// kS16: max over fluid sites of |g_i^eq| / w_i per weight class of the
// equilibrium init_eq writes (float bits into out[0..2]), and the in-place
// widening of an array's scales
hipError_t launch_eq_absmax(const InitArgs &a, unsigned int *out, hipStream_t s);
hipError_t launch_s16_rescale(void *state, const Layout &lay, uint64_t elems, const Shift16 &sh, hipStream_t s);
int step_occupancy(int codec, int variant, bool solids, bool macros);  // workgroups per CU

// Host helpers of the runtime files.  fail() records the message that
// lb_last_error returns and passes the status code through.
int fail(int code, const char *fmt, ...);
long env_long(const char *name, long dflt);  // integer environment setting (tuning knobs)

#define HIP_OR_FAIL(expr)                                                                         \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return lbm::fail(LB_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)
// Batches: variant 1 / 2 / 3 as above (always with bounce-back masks).
// lds_pad: dynamic LDS bytes per workgroup (0, or batch_cap_lds's value to
// hold the kernel to wg_cap resident workgroups per compute unit).
hipError_t launch_batch_step(int codec, int variant, const BatchArgs &a, int grid, size_t lds_pad, hipStream_t s);
size_t batch_cap_lds(int codec, int variant, int wg_cap);
hipError_t launch_batch_totals(const BatchTotalsArgs &a, hipStream_t s);
// One adjoint step; variant 1 / 2 / 3 = 4 / 2 / 1 sites per lane (FP32 storage).
hipError_t launch_adjoint(int variant, bool first, const AdjArgs &a, int grid, hipStream_t s);
int batch_occupancy(int codec, int variant, size_t lds_pad);
// Outlet flux objective: J of a stored state (one workgroup, fixed-order FP64
// sum), its seed dJ/dS_N written into a zeroed storage-layout array, and its
// direct term added to a gradient.
hipError_t launch_outlet_flux(int codec, const OutletArgs &a, hipStream_t s);
int outlet_parts(int ny, int nz);
hipError_t launch_outlet_seed(const OutletArgs &a, hipStream_t s);
hipError_t launch_outlet_direct(const OutletArgs &a, hipStream_t s);
// Raw planes (19 x n elements of esize bytes, site order) to the storage
// layout (to_state) or back.  Both pointers are device pointers.
hipError_t launch_repack(void *planes, void *state, const Layout &lay, int64_t n, int esize, bool to_state,
                         hipStream_t s);
// In-place storage: raw planes of the state S from the array (phase 1 even,
// 2 odd; flags may be nullptr), or planes into the array in the even form.
hipError_t launch_aa_planes(void *planes, void *state, const Layout &lay, int ny, int nz, const uint8_t *flags,
                            int esize, int phase, bool to_state, hipStream_t s);
// In-place steps: even (true) runs the gather-collide-push kernel, odd the local one.
hipError_t launch_aa_step(int codec, int variant, bool solids, bool from_even, const StepArgs &a, int grid,
                          hipStream_t s);
int aa_occupancy(int codec, int variant, bool solids, bool from_even);
// D2Q9: variant 1 / 2 / 3 = 4 / 2 / 1 sites per lane (FP32 storage).
hipError_t launch_step2d(int variant, bool solids, const Step2Args &a, int grid, hipStream_t s);
// D2Q9 masks (nx * ny, site order) and one dirty byte per 64 sites ((n + 63) / 64 bytes).
hipError_t launch_masks2d(const uint8_t *flags, int nx, int ny, uint32_t *nbmask, uint8_t *chunkdirty, hipStream_t s);
hipError_t launch_init2d(void *dst, const Layout &lay, int nx, int ny, const double *rho, const double *u,
                         const uint8_t *flags, hipStream_t s);
hipError_t launch_macros2d(const void *src, const Layout &lay, int nx, int ny, const uint8_t *flags, float *rho,
                           float *u, hipStream_t s);
// Raw planes (9 x n floats, site order) to a D2Q9 array (to_state) or back.
hipError_t launch_repack2d(void *planes, void *state, const Layout &lay, int64_t n, bool to_state, hipStream_t s);
int sites_per_thread(int codec, int variant);

}  // namespace lbm
