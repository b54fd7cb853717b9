// lb_pattern.hip -- lb_pattern_ms: the memory access pattern of the FP32
// one-read step with no arithmetic, timed on the device.  A measurement aid
// for the step's roofline: the rate at which HBM serves exactly this pattern
// (19 pair streams read at the pull's upstream sites and 19 written, on the
// step's tiles, chunks, workgroup-to-XCD mapping, barriers and LDS budget)
// bounds what the collide-and-stream kernel can reach.
#include <hip/hip_runtime.h>

#include <string>

#include "lb_internal.hpp"

namespace lbm {
namespace {

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

template <int TY>
__global__ __launch_bounds__(kTX * TY) void pattern_kernel(Geom g, const float* __restrict__ fin,
                                                          float* __restrict__ fout, FusedShape fs, float k) {
    using L = Lattice;
    extern __shared__ float lds_sink[];
    int x0, y0, za, zb;
    tile_of_block(fs, kTX, g.nz, x0, y0, za, zb);
    const int lane = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int x = x0 + lane, y = y0 + ty;
    const bool in = x < g.nx && y < g.ny;
    const int xc = min(x, g.nx - 1), yc = min(y, g.ny - 1);
    const size_t S = raw_stride((size_t)g.N);
    using P = typename RawPair<float>::type;
    float acc = 0.f;
    for (int z = za; z < zb; ++z) {
        P v[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int xs = wrap(xc - L::cx[i], g.nx), ys = wrap(yc - L::cy[i], g.ny), zs = wrap(z - L::cz[i], g.nz);
            v[i] = raw_pair(fin, (size_t)g.N, i, site_of(g, xs, ys, zs));
        }
        __syncthreads();
        // every store depends on every load, as after a collision (k = 0)
#pragma unroll
        for (int i = 0; i < Q; ++i) acc = fmaf(v[i].x + v[i].y, k, acc);
        if (in) {
            const size_t s = (size_t)site_of(g, xc, yc, z);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                P w = v[i];
                w.x += acc;
                __builtin_nontemporal_store(w, reinterpret_cast<P*>(fout + 2 * ((size_t)i * S + s)));
            }
        }
        __syncthreads();
    }
    if (k < -1e30f) lds_sink[threadIdx.x] = acc;  // never taken: the LDS allocation stays
}

template <int TY>
int run(const Geom& g, const FusedShape& fs, size_t lds, const float* a, float* b, hipStream_t st, int n) {
    auto kern = pattern_kernel<TY>;
    if (lds > 65536) {
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds) != hipSuccess)
            return set_error(LB_EDEVICE, "pattern_kernel LDS");
    }
    // ping-pong: even launches read a and write b, odd ones the reverse
    for (int r = 0; r < n; ++r) {
        const float* in = (r & 1) ? b : a;
        float* out = (r & 1) ? const_cast<float*>(a) : b;
        hipLaunchKernelGGL(kern, dim3(fs.nblocks), dim3(kTX * TY), lds, st, g, in, out, fs, 0.f);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(LB_EDEVICE, (std::string("pattern_kernel: ") + hipGetErrorString(e)).c_str());
    return LB_OK;
}

}  // namespace
}  // namespace lbm

using namespace lbm;

extern "C" int lb_pattern_ms(const lb_params* params, int32_t reps, double* ms) {
    std::string why;
    if (!ms) return set_error(LB_EINVAL, "ms is NULL");
    if (validate_params(params, why) != LB_OK) return set_error(LB_EINVAL, why.c_str());
    if (reps < 1) return set_error(LB_EINVAL, "reps must be >= 1");
    if (params->bc[0] || params->bc[1] || params->bc[2]) return set_error(LB_EINVAL, "periodic lattices only");
    lb_params p = *params;
    p.storage = LB_STORE_F32;
    const int TY = tile_rows(p, TILE_SINGLE);
    if (TY != kSingleTYSmall && TY != kSingleTY && TY != kSingleTYLarge)
        return set_error(LB_EINVAL, "the one-read step does not take this lattice");
    const FusedShape fs = tile_shape(p, TILE_SINGLE);
    const Geom g = make_geom(p);
    const size_t lds = tile_lds(p, TILE_SINGLE, TY);
    const size_t bytes = pop_bytes(LB_STORE_F32, (size_t)g.N);
    float *a = nullptr, *b = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = LB_OK;
    if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess)
        rc = set_error(LB_EDEVICE, "hipMalloc pattern buffers");
    if (!rc && (hipStreamCreate(&st) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
                hipEventCreate(&e1) != hipSuccess))
        rc = set_error(LB_EDEVICE, "stream or events");
    if (!rc && (hipMemsetAsync(a, 0, bytes, st) != hipSuccess || hipMemsetAsync(b, 0, bytes, st) != hipSuccess))
        rc = set_error(LB_EDEVICE, "hipMemsetAsync");
    auto launch = [&](int n) {
        switch (TY) {
            case kSingleTYSmall: return run<kSingleTYSmall>(g, fs, lds, a, b, st, n);
            case kSingleTY: return run<kSingleTY>(g, fs, lds, a, b, st, n);
            default: return run<kSingleTYLarge>(g, fs, lds, a, b, st, n);
        }
    };
    if (!rc) rc = launch(2);  // untimed
    if (!rc && hipEventRecord(e0, st) != hipSuccess) rc = set_error(LB_EDEVICE, "hipEventRecord");
    if (!rc) rc = launch(reps);
    if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = set_error(LB_EDEVICE, "hipEventRecord");
    float t = 0.f;
    if (!rc && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        rc = set_error(LB_EDEVICE, "event timing");
    if (!rc) *ms = double(t) / reps;
    if (st) (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    return rc;
}
