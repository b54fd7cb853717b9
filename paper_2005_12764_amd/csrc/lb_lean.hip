// lb_lean.hip -- instantiation and launch of the lean one-read tile kernel
// (raw FP64/FP32 storage).
#include <hip/hip_runtime.h>

#include <string>

#include "lb_internal.hpp"
#include "lb_lean.hpp"

namespace lbm {

namespace {

template <typename T, int TY, int H, bool W>
int lean_launch_h(const LatticeView& v, const T* fin, T* fout, const Coeffs<T>& c, const FusedShape& fs) {
    const size_t lds = tile_lds(*v.p, TILE_SINGLE, TY);
    auto kern = lean_kernel<T, T, TY, H, W>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return set_error(LB_EDEVICE, (std::string("lean_kernel LDS: ") + hipGetErrorString(e)).c_str());
    }
    hipLaunchKernelGGL(kern, dim3(fs.nblocks), dim3(kTX * TY), lds, v.stream, v.g, fin, fout, c, fs,
                       (const Part2<T>*)v.part_in, (Part2<T>*)v.part_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(LB_EDEVICE, (std::string("lean_kernel: ") + hipGetErrorString(e)).c_str());
    return LB_OK;
}

template <typename T, int TY, int H>
int lean_launch_w(const LatticeView& v, const T* fin, T* fout, const Coeffs<T>& c, const FusedShape& fs) {
    if (v.g.wx || v.g.wy || v.g.wz) return lean_launch_h<T, TY, H, true>(v, fin, fout, c, fs);
    return lean_launch_h<T, TY, H, false>(v, fin, fout, c, fs);
}

template <typename T, int TY>
int lean_launch_ty(const LatticeView& v, const T* fin, T* fout, const Coeffs<T>& c, const FusedShape& fs) {
    switch (tile_halo(*v.p)) {
        case 1: return lean_launch_w<T, TY, 1>(v, fin, fout, c, fs);
        case 2: return lean_launch_w<T, TY, 2>(v, fin, fout, c, fs);
        case 3: return lean_launch_w<T, TY, 3>(v, fin, fout, c, fs);
        case 4: return lean_launch_w<T, TY, 4>(v, fin, fout, c, fs);
        case 5: return lean_launch_w<T, TY, 5>(v, fin, fout, c, fs);
    }
    return set_error(LB_EINVAL, "near-contact range outside the tile kernels' halo");
}

}  // namespace

template <typename T>
int launch_lean(const LatticeView& v, const T* fin, T* fout, const Coeffs<T>& c, const FusedShape& fs) {
    // byte offsets within a buffer resource of ten arrays are 32-bit
    if ((uint64_t)kResArrays * sizeof(T) * (uint64_t)v.g.N >= ((uint64_t)1 << 32))
        return set_error(LB_EINVAL, "lattice too large for the one-read step (10 x sites x value size >= 2^32)");
    switch (fs.TY) {
        case kSingleTYSmall: return lean_launch_ty<T, kSingleTYSmall>(v, fin, fout, c, fs);
        case kSingleTY: return lean_launch_ty<T, kSingleTY>(v, fin, fout, c, fs);
        case kSingleTYLarge:
            // (FP64 rings of 16 rows do not fit the LDS: tile_rows never picks them)
            if constexpr (sizeof(T) == 4) return lean_launch_ty<T, kSingleTYLarge>(v, fin, fout, c, fs);
            break;
    }
    return set_error(LB_EINVAL, "one-read tile rows must be 4, 8 or 16 (4 or 8 in FP64)");
}

template int launch_lean<float>(const LatticeView&, const float*, float*, const Coeffs<float>&, const FusedShape&);
template int launch_lean<double>(const LatticeView&, const double*, double*, const Coeffs<double>&,
                                 const FusedShape&);

}  // namespace lbm
