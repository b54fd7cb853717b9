// lb_noalloc.hip -- lb_state_totals_noalloc: the compensated totals of
// lb_moments for a population state the caller holds, without any device
// allocation (the per-block partial sums live in a static device array).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "lb_internal.hpp"

namespace lbm {

// Populations f^r_i, f^b_i of a caller state in the layout of lb_get_state
// ([2][19][N], post-streaming), read at their own sites as shifted variables.
template <typename T>
struct PlainPop {
    const T* f;
    size_t N;
    template <typename R>
    __device__ __forceinline__ void pull(const Geom&, int s, int, int, int, R (&t)[Q], R (&d)[Q]) const {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const R fr = R(f[(size_t)i * N + s]), fb = R(f[(size_t)(Q + i) * N + s]);
            t[i] = (fr + fb) - weight<R>(i);
            d[i] = fr - fb;
        }
    }
};

}  // namespace lbm

using namespace lbm;

namespace {

// Workgroups of the totals kernel and the scratch they fill: one compensated
// pair per total per workgroup (kTotalsBlocks x 7 x 16 B = 57,344 B per device).
constexpr int kNoallocBlocks = kTotalsBlocks;
__device__ __align__(256) Neu scratch[kNoallocBlocks * NTOT];

// Device address of `scratch` per device (the array's name is a host-side
// stand-in in host code; each device holds its own copy).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_of(int dev, Neu** out) {
    if (dev < 0 || dev >= kMaxDevices) return set_error(LB_EDEVICE, "device index outside the library's table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return set_error(LB_EDEVICE, (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
        g_scratch_ptr[dev] = ptr;
    }
    *out = (Neu*)g_scratch_ptr[dev];
    return LB_OK;
}

}  // namespace

extern "C" {

int lb_state_totals_noalloc(const lb_params* params, const void* f, int32_t dtype, double* totals,
                            void* hip_stream) {
    if (!params || !f || !totals) return set_error(LB_EINVAL, "NULL argument");
    if (params->nx < 1 || params->ny < 1 || params->nz < 1) return set_error(LB_EINVAL, "lattice sizes must be >= 1");
    const double n = double(params->nx) * double(params->ny) * double(params->nz);
    if (n >= 2147483647.0) return set_error(LB_EINVAL, "lattice too large (sites must fit in 31 bits)");
    if (dtype != LB_DTYPE_F64 && dtype != LB_DTYPE_F32)
        return set_error(LB_EINVAL, "dtype must be LB_DTYPE_F64 or LB_DTYPE_F32");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(LB_EDEVICE, "no current HIP device");
    Neu* part = nullptr;
    int rc = scratch_of(dev, &part);
    if (rc) return rc;
    Geom g{};
    g.nx = params->nx;
    g.ny = params->ny;
    g.nz = params->nz;
    g.nxy = g.nx * g.ny;
    g.N = g.nxy * g.nz;
    const hipStream_t st = (hipStream_t)hip_stream;
    const unsigned grid = (unsigned)std::min<long long>(kNoallocBlocks, ((long long)g.N + 255) / 256);
    // every workgroup writes its own partials: nothing in scratch needs clearing
    if (dtype == LB_DTYPE_F64)
        hipLaunchKernelGGL((totals_kernel<double, PlainPop<double>>), dim3(grid), dim3(256), 0, st, g,
                           PlainPop<double>{(const double*)f, (size_t)g.N}, part);
    else
        hipLaunchKernelGGL((totals_kernel<double, PlainPop<float>>), dim3(grid), dim3(256), 0, st, g,
                           PlainPop<float>{(const float*)f, (size_t)g.N}, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(LB_EDEVICE, (std::string("totals_kernel: ") + hipGetErrorString(e)).c_str());
    hipLaunchKernelGGL(totals_final_kernel, dim3(1), dim3(256), 0, st, (const Neu*)part, (int)grid, totals);
    e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(LB_EDEVICE, (std::string("totals_final_kernel: ") + hipGetErrorString(e)).c_str());
    return LB_OK;
}

}  // extern "C"
