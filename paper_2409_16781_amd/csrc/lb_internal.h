// Internal interface between the host runtime (lb_capi.hip) and the kernels
// (lb_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int kQ = 19;
constexpr int kBlock = 256;        // threads per workgroup of every lattice kernel
constexpr int kRingCap = 4096;     // per-step conservation totals kept on the device

enum Codec : int { kF32 = 0, kF16 = 1, kBF16 = 2 };

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

// Everything one step launch needs.  Pointers are device pointers.
struct StepArgs {
    const void *src;          // stored state (post-collision of the previous step), plane 0
    void *dst;                // new state, plane 0
    uint64_t plane;           // elements between consecutive population planes (>= N)
    int nx, ny, nz;
    int nslots;               // N / sites_per_thread
    FastDiv div_nx, div_ny;
    float omega;
    float fx, fy, fz;
    const uint32_t *nbmask;   // per site: bit i = site x - c_i is solid, bit 31 = site is solid
    const uint8_t *rowdirty;  // per row (y, z): 1 if any site of the row has bit set in nbmask
    float *rho_out;           // optional macros output (N floats) or nullptr
    float *u_out;             // optional macros output (3N floats) or nullptr
    double *partials;         // 4 doubles per workgroup
    unsigned int *ticket;     // workgroup arrival counter, 0 between launches
    double *ring;             // kRingCap x 4 doubles
    unsigned long long *step_counter;
    double n_fluid;           // number of fluid sites (exact in a double)
};

struct InitArgs {
    void *dst;
    uint64_t plane;
    int n;                    // N
    const double *rho;        // N or nullptr
    const double *u;          // 3N or nullptr
    const uint8_t *flags;     // device flags or nullptr
};

struct MacroArgs {
    const void *src;
    uint64_t plane;
    int n;
    float fx, fy, fz;
    const uint8_t *flags;
    float *rho;
    float *u;
};

// Launchers (lb_kernels.hip).  variant: 0 = one site per thread; 1 / 2 / 3 = vector
// rows with 16- / 8- / 4-byte accesses per lane and population plane.
hipError_t launch_step(int codec, int variant, bool solids, bool macros, const StepArgs &a, int grid,
                       hipStream_t s);
hipError_t launch_init(int codec, const InitArgs &a, hipStream_t s);
hipError_t launch_macros(int codec, const MacroArgs &a, hipStream_t s);
hipError_t launch_masks(const uint8_t *flags, int nx, int ny, int nz, uint32_t *nbmask, uint8_t *rowdirty,
                        hipStream_t s);
hipError_t launch_zero_solid_macros(const uint8_t *flags, int n, float *rho, float *u, hipStream_t s);
hipError_t launch_copy(const void *src, void *dst, uint64_t bytes, hipStream_t s);
int step_occupancy(int codec, int variant, bool solids, bool macros);  // workgroups per CU
int sites_per_thread(int codec, int variant);

}  // namespace lbm
