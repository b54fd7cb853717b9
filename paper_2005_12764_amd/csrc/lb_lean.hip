// lb_lean.hip -- instantiation and launch of the lean one-read tile kernel for
// raw (FP64/FP32) storage.
#include "lb_lean_launch.hpp"

namespace lbm {

template <typename T>
int launch_lean(const LatticeView& v, const T* fin, T* fout, const Coeffs<T>& c, const FusedShape& fs) {
    // byte offsets within a buffer resource of five pair arrays are 32-bit
    if ((uint64_t)kResArrays * sizeof(T) * (uint64_t)raw_stride((size_t)v.g.N) >= ((uint64_t)1 << 32))
        return set_error(LB_EINVAL, "lattice too large for the one-read step (10 x sites x value size >= 2^32)");
    const LeanRaw<T> st{fin, fout};
    switch (fs.TY) {
        case kSingleTYSmall: return lean_launch::launch_ty<LeanRaw<T>, kSingleTYSmall>(v, st, c, fs);
        case kSingleTY: return lean_launch::launch_ty<LeanRaw<T>, kSingleTY>(v, st, c, fs);
        case kSingleTYLarge:
            // (FP64 rings of 16 rows do not fit the LDS: tile_rows never picks them)
            if constexpr (sizeof(T) == 4) return lean_launch::launch_ty<LeanRaw<T>, kSingleTYLarge>(v, st, c, fs);
            break;
    }
    return set_error(LB_EINVAL, "one-read tile rows must be 4, 8 or 16 (4 or 8 in FP64)");
}

template int launch_lean<float>(const LatticeView&, const float*, float*, const Coeffs<float>&, const FusedShape&);
template int launch_lean<double>(const LatticeView&, const double*, double*, const Coeffs<double>&,
                                 const FusedShape&);

}  // namespace lbm
