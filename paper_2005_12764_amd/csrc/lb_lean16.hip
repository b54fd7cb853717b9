// lb_lean16.hip -- instantiation and launch of the lean one-read tile kernel
// for the 16-bit moment-split storage (fp16, bf16).
#include "lb_lean_launch.hpp"

namespace lbm {

template <typename H>
int launch_lean_split(const LatticeView& v, const SplitPop<H>& src, const SplitPop<H>& dst, const Coeffs<float>& c,
                      const FusedShape& fs) {
    // byte offsets within the record and deviation resources are 32-bit
    if ((uint64_t)32 * (uint64_t)v.g.N >= ((uint64_t)1 << 32) || (uint64_t)2 * Q * (uint64_t)dev_stride((size_t)v.g.N) >= ((uint64_t)1 << 32))
        return set_error(LB_EINVAL, "lattice too large for the one-read step of 16-bit storage");
    LeanSplit<H> st;
    st.rin = src.rec;
    st.din = src.dev;
    st.rout = dst.rec;
    st.dout = dst.dev;
    st.codec = src;
    st.ring = nullptr;
    st.TY = fs.TY;
    switch (fs.TY) {
        case kSingleTYSmall: return lean_launch::launch_ty<LeanSplit<H>, kSingleTYSmall>(v, st, c, fs);
        case kSingleTY: return lean_launch::launch_ty<LeanSplit<H>, kSingleTY>(v, st, c, fs);
    }
    return set_error(LB_EINVAL, "one-read tile rows of 16-bit storage must be 4 or 8");
}

template int launch_lean_split<__half>(const LatticeView&, const SplitPop<__half>&, const SplitPop<__half>&,
                                       const Coeffs<float>&, const FusedShape&);
template int launch_lean_split<__hip_bfloat16>(const LatticeView&, const SplitPop<__hip_bfloat16>&,
                                               const SplitPop<__hip_bfloat16>&, const Coeffs<float>&,
                                               const FusedShape&);

}  // namespace lbm
