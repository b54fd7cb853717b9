// lb_lean_launch.hpp -- host-side launch of the lean one-read tile kernel for
// a storage policy (shared by the translation units that instantiate it).
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "lb_internal.hpp"
#include "lb_lean.hpp"

namespace lbm {
namespace lean_launch {

template <typename S, int TY, int HALO, bool W, bool MV>
int launch_h(const LatticeView& v, const S& st, const Coeffs<typename S::R>& c, const FusedShape& fs) {
    using R = typename S::R;
    const size_t lds = lean_lds_bytes<S, TY, HALO>();
    auto kern = lean_kernel<S, TY, HALO, W, MV>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return set_error(LB_EDEVICE, (std::string("lean_kernel LDS: ") + hipGetErrorString(e)).c_str());
    }
    // the next step's pull adds moving-wall terms even when this one (the
    // first after a state was set) does not: the gathered sums follow the next
    const int moving_next = make_geom(*v.p).moving;
    hipLaunchKernelGGL(kern, dim3(fs.nblocks), dim3(kTX * TY), lds, v.stream, v.g, st, c, fs,
                       (const Part2<R>*)v.part_in, (Part2<R>*)v.part_out, moving_next);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(LB_EDEVICE, (std::string("lean_kernel: ") + hipGetErrorString(e)).c_str());
    return LB_OK;
}

template <typename S, int TY, int HALO>
int launch_w(const LatticeView& v, const S& st, const Coeffs<typename S::R>& c, const FusedShape& fs) {
    // walls at rest and moving walls take separate instantiations (the
    // resting-wall kernel holds none of the wall-term code)
    if (v.g.moving || make_geom(*v.p).moving) return launch_h<S, TY, HALO, true, true>(v, st, c, fs);
    if (v.g.wx || v.g.wy || v.g.wz) return launch_h<S, TY, HALO, true, false>(v, st, c, fs);
    return launch_h<S, TY, HALO, false, false>(v, st, c, fs);
}

template <typename S, int TY>
int launch_ty(const LatticeView& v, const S& st, const Coeffs<typename S::R>& c, const FusedShape& fs) {
    switch (tile_halo(*v.p)) {
        case 1: return launch_w<S, TY, 1>(v, st, c, fs);
        case 2: return launch_w<S, TY, 2>(v, st, c, fs);
        case 3: return launch_w<S, TY, 3>(v, st, c, fs);
        case 4: return launch_w<S, TY, 4>(v, st, c, fs);
        case 5: return launch_w<S, TY, 5>(v, st, c, fs);
    }
    return set_error(LB_EINVAL, "near-contact range outside the tile kernels' halo");
}

}  // namespace lean_launch
}  // namespace lbm
