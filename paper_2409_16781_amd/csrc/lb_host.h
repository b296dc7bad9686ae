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

}  // namespace lbm
