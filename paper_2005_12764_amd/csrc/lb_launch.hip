// lb_launch.hip -- kernel instantiation and dispatch over storage types.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <type_traits>

#include "lb_internal.hpp"

namespace lbm {

namespace {

constexpr int kBlock = 256;

int launch_status(const char* what) {
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) return LB_OK;
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return set_error(LB_EDEVICE, m.c_str());
}

unsigned grid_for(int N) { return (unsigned)((N + kBlock - 1) / kBlock); }

template <typename H>
SplitPop<H> split_view(void* buf, size_t N, int scale_log2) {
    SplitPop<H> s;
    s.rec = (float*)buf;
    s.dev = (H*)((float*)buf + 8 * N);
    s.N = N;
    const float sc = std::is_same<H, __half>::value ? std::ldexp(1.0f, scale_log2) : 1.0f;
    s.scale = sc;
    s.inv_scale = 1.0f / sc;
    return s;
}

// Calls fn(R{}, src, coeffs) with the compute type and a view of the current
// state in its storage.
template <typename Fn>
int with_state(const LatticeView& v, Fn&& fn) {
    const size_t N = (size_t)v.g.N;
    switch (v.p->storage) {
        case LB_STORE_F64: return fn(double(0), RawPop<double>{(double*)v.cur, N}, v.cd);
        case LB_STORE_F32: return fn(float(0), RawPop<float>{(float*)v.cur, N}, v.cf);
        case LB_STORE_F16:
            if (v.pending) return fn(float(0), RawPop<float>{(float*)v.pending, N}, v.cf);
            return fn(float(0), split_view<__half>(v.cur, N, v.p->scale_log2), v.cf);
        case LB_STORE_BF16:
            if (v.pending) return fn(float(0), RawPop<float>{(float*)v.pending, N}, v.cf);
            return fn(float(0), split_view<__hip_bfloat16>(v.cur, N, v.p->scale_log2), v.cf);
    }
    return set_error(LB_EINVAL, "unknown storage");
}

template <typename R, typename Src, typename Dst>
int two_pass(const LatticeView& v, const Src& src, const Dst& dst, const Coeffs<R>& c, const StepEvents* t) {
    const unsigned grid = grid_for(v.g.N);
    if (t) (void)hipEventRecord(t->ev[0], v.stream);
    hipLaunchKernelGGL((phase_kernel<R, Src>), dim3(grid), dim3(kBlock), 0, v.stream, v.g, src, (R*)v.phi);
    int rc = launch_status("phase_kernel");
    if (rc) return rc;
    if (t) (void)hipEventRecord(t->ev[1], v.stream);
    hipLaunchKernelGGL((collide_kernel<R, Src, Dst>), dim3(grid), dim3(kBlock), 0, v.stream, v.g, src, dst,
                       (const R*)v.phi, c);
    rc = launch_status("collide_kernel");
    if (t) (void)hipEventRecord(t->ev[2], v.stream);
    return rc;
}

}  // namespace

int choose_kernel(const lb_params& p) {
    (void)p;
    return LB_KERNEL_TWOPASS;
}

int launch_step(const LatticeView& v, int kernel, const StepEvents* t) {
    (void)kernel;
    const size_t N = (size_t)v.g.N;
    switch (v.p->storage) {
        case LB_STORE_F64: {
            RawPop<double> dst{(double*)v.nxt, N};
            return with_state(v, [&](auto rt, auto src, const auto& c) {
                using R = decltype(rt);
                if constexpr (std::is_same<R, double>::value) return two_pass<R>(v, src, dst, c, t);
                return set_error(LB_EINVAL, "storage/compute mismatch");
            });
        }
        case LB_STORE_F32: {
            RawPop<float> dst{(float*)v.nxt, N};
            return with_state(v, [&](auto rt, auto src, const auto& c) {
                using R = decltype(rt);
                if constexpr (std::is_same<R, float>::value) return two_pass<R>(v, src, dst, c, t);
                return set_error(LB_EINVAL, "storage/compute mismatch");
            });
        }
        case LB_STORE_F16: {
            auto dst = split_view<__half>(v.nxt, N, v.p->scale_log2);
            return with_state(v, [&](auto rt, auto src, const auto& c) {
                using R = decltype(rt);
                if constexpr (std::is_same<R, float>::value) return two_pass<R>(v, src, dst, c, t);
                return set_error(LB_EINVAL, "storage/compute mismatch");
            });
        }
        case LB_STORE_BF16: {
            auto dst = split_view<__hip_bfloat16>(v.nxt, N, v.p->scale_log2);
            return with_state(v, [&](auto rt, auto src, const auto& c) {
                using R = decltype(rt);
                if constexpr (std::is_same<R, float>::value) return two_pass<R>(v, src, dst, c, t);
                return set_error(LB_EINVAL, "storage/compute mismatch");
            });
        }
    }
    return set_error(LB_EINVAL, "unknown storage");
}

// Initial state goes to raw storage: the current buffer for F64/F32, the
// pending FP32 buffer for 16-bit lattices.
template <typename In>
static int init_typed(const LatticeView& v, const In* rr, const In* rb, const In* u) {
    const unsigned grid = grid_for(v.g.N);
    if (v.p->storage == LB_STORE_F64) {
        hipLaunchKernelGGL((init_raw_kernel<double, In>), dim3(grid), dim3(kBlock), 0, v.stream, v.g,
                           (double*)v.cur, rr, rb, u);
    } else {
        float* dst = (float*)(v.p->storage == LB_STORE_F32 ? v.cur : v.pending);
        hipLaunchKernelGGL((init_raw_kernel<float, In>), dim3(grid), dim3(kBlock), 0, v.stream, v.g, dst, rr, rb, u);
    }
    return launch_status("init_raw_kernel");
}

int launch_init(const LatticeView& v, const void* rr, const void* rb, const void* u, int dtype) {
    if (dtype == LB_DTYPE_F64) return init_typed<double>(v, (const double*)rr, (const double*)rb, (const double*)u);
    return init_typed<float>(v, (const float*)rr, (const float*)rb, (const float*)u);
}

template <typename In>
static int import_typed(const LatticeView& v, const In* f) {
    const unsigned grid = grid_for(v.g.N);
    if (v.p->storage == LB_STORE_F64) {
        hipLaunchKernelGGL((import_raw_kernel<double, In>), dim3(grid), dim3(kBlock), 0, v.stream, v.g,
                           (double*)v.cur, f);
    } else {
        float* dst = (float*)(v.p->storage == LB_STORE_F32 ? v.cur : v.pending);
        hipLaunchKernelGGL((import_raw_kernel<float, In>), dim3(grid), dim3(kBlock), 0, v.stream, v.g, dst, f);
    }
    return launch_status("import_raw_kernel");
}

int launch_import(const LatticeView& v, const void* f, int dtype) {
    if (dtype == LB_DTYPE_F64) return import_typed<double>(v, (const double*)f);
    return import_typed<float>(v, (const float*)f);
}

int launch_export(const LatticeView& v, void* out, int dtype) {
    const unsigned grid = grid_for(v.g.N);
    return with_state(v, [&](auto rt, auto src, const auto&) {
        using R = decltype(rt);
        using S = decltype(src);
        if (dtype == LB_DTYPE_F64)
            hipLaunchKernelGGL((export_kernel<R, S, double>), dim3(grid), dim3(kBlock), 0, v.stream, v.g, src, (double*)out);
        else
            hipLaunchKernelGGL((export_kernel<R, S, float>), dim3(grid), dim3(kBlock), 0, v.stream, v.g, src, (float*)out);
        return launch_status("export_kernel");
    });
}

int launch_moments(const LatticeView& v, void* rr, void* rb, void* j, int dtype) {
    const unsigned grid = grid_for(v.g.N);
    return with_state(v, [&](auto rt, auto src, const auto&) {
        using R = decltype(rt);
        using S = decltype(src);
        if (dtype == LB_DTYPE_F64)
            hipLaunchKernelGGL((moments_kernel<R, S, double>), dim3(grid), dim3(kBlock), 0, v.stream, v.g, src,
                               (double*)rr, (double*)rb, (double*)j);
        else
            hipLaunchKernelGGL((moments_kernel<R, S, float>), dim3(grid), dim3(kBlock), 0, v.stream, v.g, src,
                               (float*)rr, (float*)rb, (float*)j);
        return launch_status("moments_kernel");
    });
}

int launch_totals(const LatticeView& v, Neu* partial, double* dtot) {
    const unsigned grid = (unsigned)std::min<int>(kTotalsBlocks, (int)grid_for(v.g.N));
    int rc = with_state(v, [&](auto rt, auto src, const auto&) {
        using R = decltype(rt);
        using S = decltype(src);
        hipLaunchKernelGGL((totals_kernel<R, S>), dim3(grid), dim3(kBlock), 0, v.stream, v.g, src, partial);
        return launch_status("totals_kernel");
    });
    if (rc) return rc;
    hipLaunchKernelGGL(totals_final_kernel, dim3(1), dim3(kBlock), 0, v.stream, partial, (int)grid, dtot);
    return launch_status("totals_final_kernel");
}

}  // namespace lbm
