// Host-side helpers of the runtime sources (no device code).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

namespace lbm {

// HIP events of one timing call, destroyed on every return path.
struct Events {
    std::vector<hipEvent_t> ev;
    explicit Events(size_t n) : ev(n, nullptr) {}
    Events(const Events &) = delete;
    Events &operator=(const Events &) = delete;
    hipError_t create()
    {
        for (auto &e : ev) {
            const hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) {
                e = nullptr;
                return r;
            }
        }
        return hipSuccess;
    }
    ~Events()
    {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    hipEvent_t operator[](size_t k) const { return ev[k]; }
};

// Captured runs of one length: one graph per start parity (a run of odd
// length ends on the other parity, so successive replays alternate).  The
// owner calls invalidate() whenever a launch argument changes.
struct RunGraphs {
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    int len = 0;
    hipStream_t cap = nullptr;  // capture stream, created on first use
    void invalidate()
    {
        for (auto &e : exec)
            if (e) {
                (void)hipGraphExecDestroy(e);
                e = nullptr;
            }
        len = 0;
    }
    void release()
    {
        invalidate();
        if (cap) (void)hipStreamDestroy(cap);
        cap = nullptr;
    }
};

}  // namespace lbm
