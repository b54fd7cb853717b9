// lb_launch.hip -- kernel instantiation and dispatch over storage types.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <string>
#include <type_traits>

#include "lb_internal.hpp"
#include "lb_korteweg.hpp"
#include "lb_lean.hpp"
#include "lb_shanchen.hpp"
#include "lb_single.hpp"

namespace lbm {

namespace {

constexpr int kBlock = 256;
int max_lds_bytes();
int device_lds_bytes();
size_t real_size(const lb_params& p);
bool split_storage(const lb_params& p);

int launch_status(const char* what) {
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) return LB_OK;
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return set_error(LB_EDEVICE, m.c_str());
}

unsigned grid_for(int N) { return (unsigned)((N + kBlock - 1) / kBlock); }

template <typename H, bool MW = false>
SplitPop<H, MW> split_view(void* buf, size_t N, int scale_log2) {
    SplitPop<H, MW> s;
    s.rec = (float*)buf;
    s.dev = (H*)((float*)buf + 8 * N);
    s.N = N;
    const float sc = std::is_same<H, __half>::value ? std::ldexp(1.0f, scale_log2) : 1.0f;
    s.scale = sc;
    s.inv_scale = 1.0f / sc;
    return s;
}

// Calls fn(R{}, src, coeffs) with the compute type and a view of the current
// state in its storage; lattices with moving walls get the storage types that
// add the moving-wall terms (a raw initial state is never pulled with them).
template <bool MW, typename Fn>
int with_state_mw(const LatticeView& v, Fn&& fn) {
    const size_t N = (size_t)v.g.N;
    switch (v.p->storage) {
        case LB_STORE_F64: return fn(double(0), RawPop<double, MW>{(double*)v.cur, N}, v.cd);
        case LB_STORE_F32: return fn(float(0), RawPop<float, MW>{(float*)v.cur, N}, v.cf);
        case LB_STORE_F16:
            if (v.pending) return fn(float(0), RawPop<float>{(float*)v.pending, N}, v.cf);
            return fn(float(0), split_view<__half, MW>(v.cur, N, v.p->scale_log2), v.cf);
        case LB_STORE_BF16:
            if (v.pending) return fn(float(0), RawPop<float>{(float*)v.pending, N}, v.cf);
            return fn(float(0), split_view<__hip_bfloat16, MW>(v.cur, N, v.p->scale_log2), v.cf);
    }
    return set_error(LB_EINVAL, "unknown storage");
}

template <typename Fn>
int with_state(const LatticeView& v, Fn&& fn) {
    if (v.g.moving) return with_state_mw<true>(v, fn);
    return with_state_mw<false>(v, fn);
}

// LDS per workgroup the device allows (160 KiB on gfx950).
int device_lds_bytes() {
    static int cached = -1;
    if (cached < 0) {
        int dev = 0, v = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 65536;
        cached = v;
    }
    return cached;
}

// Budget of the two-pass tile kernels (64 KiB: more LDS per workgroup would
// cost them occupancy).
int max_lds_bytes() { return std::min(device_lds_bytes(), 65536); }

size_t real_size(const lb_params& p) { return p.storage == LB_STORE_F64 ? 8 : 4; }

bool split_storage(const lb_params& p) { return p.storage >= LB_STORE_F16; }

// Collide pass of the two-pass step: z-marching tiles reading the phase
// pass's phi through an LDS ring.
template <typename R, typename Src, typename Dst, int H>
int zmarch_h(const LatticeView& v, const Src& src, const Dst& dst, const Coeffs<R>& c, const R* phi_in) {
    const FusedShape fs = tile_shape(*v.p, TILE_COLLIDE);
    const size_t lds = tile_lds(*v.p, TILE_COLLIDE, fs.TY);
    hipLaunchKernelGGL((fused_kernel<R, Src, Dst, kTX, H>), dim3(fs.nblocks), dim3(kBlock), lds, v.stream, v.g, src,
                       dst, c, fs, phi_in);
    return launch_status("collide pass");
}

template <typename R, typename Src, typename Dst>
int zmarch(const LatticeView& v, const Src& src, const Dst& dst, const Coeffs<R>& c, const R* phi_in) {
    switch (tile_halo(*v.p)) {
        case 1: return zmarch_h<R, Src, Dst, 1>(v, src, dst, c, phi_in);
        case 2: return zmarch_h<R, Src, Dst, 2>(v, src, dst, c, phi_in);
        case 3: return zmarch_h<R, Src, Dst, 3>(v, src, dst, c, phi_in);
        case 4: return zmarch_h<R, Src, Dst, 4>(v, src, dst, c, phi_in);
        case 5: return zmarch_h<R, Src, Dst, 5>(v, src, dst, c, phi_in);
    }
    return set_error(LB_EINVAL, "near-contact range outside the tile kernels' halo");
}

// One-read step: the own partial sums of the current state (and phi where
// they are complete) come from the previous one-read step, or from
// part_kernel when no such step made them; assemble_kernel adds the
// cross-tile terms into phi of the face sites; the tile kernel collides,
// streams and gathers the next state's sums and interior phi.
template <typename R, typename Src, typename Dst, int TY, int H>
int single_h(const LatticeView& v, const Src& src, const Dst& dst, const Coeffs<R>& c, const FusedShape& fs) {
    if constexpr (!Src::ring && !Dst::ring) {
        // raw storage: the lean tile kernel
        return launch_lean<R>(v, src.f, dst.f, c, fs);
    } else if constexpr (Src::ring && Dst::ring) {
        // 16-bit moment-split storage: the lean tile kernel with the record ring
        return launch_lean_split(v, src, dst, c, fs);
    } else {
        // the first step of a 16-bit lattice, from its raw FP32 initial state
        const size_t lds = tile_lds(*v.p, TILE_SINGLE, TY);
        auto kern = single_kernel<R, Src, Dst, kTX, TY, H>;
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess)
                return set_error(LB_EDEVICE, (std::string("single_kernel LDS: ") + hipGetErrorString(e)).c_str());
        }
        hipLaunchKernelGGL(kern, dim3(fs.nblocks), dim3(kTX * TY), lds, v.stream, v.g, src, dst, c, fs,
                           (const Part2<R>*)v.part_in, (Part2<R>*)v.part_out);
        return launch_status("single_kernel");
    }
}

// phi of the face sites of a one-read state (its interior phi is already in
// the phase-sum buffer).
template <typename R, typename Src, int TY>
int assemble_phase(const LatticeView& v, const Src& src, const FusedShape& fs) {
    const FaceSet faces = face_set(v.g, kTX, TY, fs.TZ);
    hipLaunchKernelGGL((assemble_kernel<R, Src, kTX, TY>), dim3(grid_for(faces.row_sites + faces.edge_sites)),
                       dim3(kBlock), 0, v.stream, v.g, src, faces, (Part2<R>*)v.part_in);
    return launch_status("assemble_kernel");
}

template <typename R, typename Src, typename Dst, int TY>
int single_ty(const LatticeView& v, const Src& src, const Dst& dst, const Coeffs<R>& c, const FusedShape& fs,
              const StepEvents* t) {
    if (!v.part_valid) {
        hipLaunchKernelGGL((part_kernel<R, Src, kTX, TY>), dim3(grid_for(v.g.N)), dim3(kBlock), 0, v.stream, v.g,
                           src, fs.TZ, (Part2<R>*)v.part_in);
        int rc = launch_status("part_kernel");
        if (rc) return rc;
    }
    int rc = assemble_phase<R, Src, TY>(v, src, fs);
    if (rc) return rc;
    if (t) (void)hipEventRecord(t->ev[1], v.stream);
    switch (tile_halo(*v.p)) {
        case 1: return single_h<R, Src, Dst, TY, 1>(v, src, dst, c, fs);
        case 2: return single_h<R, Src, Dst, TY, 2>(v, src, dst, c, fs);
        case 3: return single_h<R, Src, Dst, TY, 3>(v, src, dst, c, fs);
        case 4: return single_h<R, Src, Dst, TY, 4>(v, src, dst, c, fs);
        case 5: return single_h<R, Src, Dst, TY, 5>(v, src, dst, c, fs);
    }
    return set_error(LB_EINVAL, "near-contact range outside the tile kernels' halo");
}

template <typename R, typename Src, typename Dst>
int single_pass(const LatticeView& v, const Src& src, const Dst& dst, const Coeffs<R>& c, const StepEvents* t) {
    if (!v.part_in || !v.part_out) return set_error(LB_EINVAL, "one-read step without its phase buffers");
    const FusedShape fs = v.shape_set ? v.shape : tile_shape(*v.p, TILE_SINGLE);
    if (t) (void)hipEventRecord(t->ev[0], v.stream);
    int rc;
    if (fs.TY == kSingleTY) rc = single_ty<R, Src, Dst, kSingleTY>(v, src, dst, c, fs, t);
    else if (fs.TY == kSingleTYSmall) rc = single_ty<R, Src, Dst, kSingleTYSmall>(v, src, dst, c, fs, t);
    else if (fs.TY == kSingleTYLarge) rc = single_ty<R, Src, Dst, kSingleTYLarge>(v, src, dst, c, fs, t);
    else return set_error(LB_EINVAL, "one-read tile does not fit in LDS");
    if (rc) return rc;
    if (t) (void)hipEventRecord(t->ev[2], v.stream);
    return LB_OK;
}

// Phase pass: raw storage pulls site by site; 16-bit moment-split storage
// runs z-marching tiles with the source records staged in LDS.
template <typename R, typename Src>
int phase_pass(const LatticeView& v, const Src& src) {
    if constexpr (Src::ring) {
        if (tile_rows(*v.p, TILE_PHASE) > 0) {
            const FusedShape fs = tile_shape(*v.p, TILE_PHASE);
            hipLaunchKernelGGL((phase_tile_kernel<R, Src, kTX>), dim3(fs.nblocks), dim3(kBlock),
                               tile_lds(*v.p, TILE_PHASE, fs.TY), v.stream, v.g, src, (R*)v.phi, fs);
            return launch_status("phase_tile_kernel");
        }
    }
    hipLaunchKernelGGL((phase_kernel<R, Src>), dim3(grid_for(v.g.N)), dim3(kBlock), 0, v.stream, v.g, src, (R*)v.phi);
    return launch_status("phase_kernel");
}

// Two passes: the phase pass writes phi; the collide pass z-marches tiles
// with phi in an LDS ring (or, when the ring does not fit, reads phi from
// global memory site by site).
// Shan-Chen step (raw storage): density pass, then the collide tiles with the
// density pairs in an LDS ring.
template <typename R, typename Src, typename Dst>
int sc_two_pass(const LatticeView& v, const Src& src, const Dst& dst, const Coeffs<R>& c, const StepEvents* t) {
    if constexpr (Src::ring || Dst::ring) {
        return set_error(LB_EINVAL, "the Shan-Chen model needs raw storage");
    } else {
        if (t) (void)hipEventRecord(t->ev[0], v.stream);
        RhoPair<R>* rho2 = (RhoPair<R>*)v.phi;
        hipLaunchKernelGGL((sc_density_kernel<R, Src>), dim3(grid_for(v.g.N)), dim3(kBlock), 0, v.stream, v.g, src,
                           rho2);
        int rc = launch_status("sc_density_kernel");
        if (rc) return rc;
        if (t) (void)hipEventRecord(t->ev[1], v.stream);
        const FusedShape fs = tile_shape(*v.p, TILE_COLLIDE);
        const size_t lds = sc_ring_bytes<R>(fs.TY, kTX);
        hipLaunchKernelGGL((sc_collide_kernel<R, Src, Dst, kTX>), dim3(fs.nblocks), dim3(kBlock), lds, v.stream, v.g,
                           src, dst, c, fs, (const RhoPair<R>*)rho2);
        rc = launch_status("sc_collide_kernel");
        if (t) (void)hipEventRecord(t->ev[2], v.stream);
        return rc;
    }
}

template <typename R, typename Src, typename Dst>
int two_pass(const LatticeView& v, const Src& src, const Dst& dst, const Coeffs<R>& c, const StepEvents* t) {
    if (!v.phi) return set_error(LB_EINVAL, "two-pass step without a phase-field buffer");
    if (v.p->model == LB_MODEL_SHAN_CHEN) return sc_two_pass<R>(v, src, dst, c, t);
    if (t) (void)hipEventRecord(t->ev[0], v.stream);
    int rc = phase_pass<R>(v, src);
    if (rc) return rc;
    if (t) (void)hipEventRecord(t->ev[1], v.stream);
    if (tile_rows(*v.p, TILE_COLLIDE) > 0) {
        rc = zmarch<R>(v, src, dst, c, (const R*)v.phi);
    } else {
        hipLaunchKernelGGL((collide_kernel<R, Src, Dst>), dim3(grid_for(v.g.N)), dim3(kBlock), 0, v.stream, v.g, src,
                           dst, (const R*)v.phi, c);
        rc = launch_status("collide_kernel");
    }
    if (t) (void)hipEventRecord(t->ev[2], v.stream);
    return rc;
}

template <typename R, typename Src, typename Dst>
int step_with(const LatticeView& v, int kernel, const Src& src, const Dst& dst, const Coeffs<R>& c,
              const StepEvents* t) {
    if constexpr (!Src::moving) {
        if (kernel == LB_KERNEL_FUSED) return single_pass<R>(v, src, dst, c, t);
    }
    return two_pass<R>(v, src, dst, c, t);
}

}  // namespace

int env_int(const char* name, int dflt) {
    const char* e = std::getenv(name);
    return (e && *e) ? std::atoi(e) : dflt;
}

namespace {
TileSetting g_tiles[4][4] = {};  // [kind][storage]
}  // namespace

TileSetting tile_setting(int kind, int storage) {
    if (kind < 0 || kind > 3 || storage < 0 || storage > 3) return TileSetting{0, 0};
    return g_tiles[kind][storage];
}
void set_tile_setting(int kind, int storage, int ty, int tz) { g_tiles[kind][storage] = TileSetting{ty, tz}; }

int tile_halo(const lb_params& p) {
    return 1 + ((p.nc_strength > 0.0 && p.model == LB_MODEL_COLOUR_GRADIENT) ? p.nc_range : 0);
}

size_t tile_lds(const lb_params& p, int kind, int TY) {
    const int H = tile_halo(p);
    const size_t phi = (size_t)(2 * H + 1) * (TY + 2 * H) * (kTX + 2 * H) * real_size(p);
    const size_t rec = (size_t)3 * (TY + 2) * (kTX + 2) * 32;
    const bool split = split_storage(p);
    switch (kind) {
        case TILE_PHASE: return rec;
        case TILE_COLLIDE: return ((phi + 15) & ~size_t(15)) + (split ? rec : 0);
        default:  // TILE_SINGLE: phi ring, record ring, exchange of the c_y != 0 directions
                  // (raw storage: rows padded by a zero at both ends), running x-face sums
                  // of the edge lanes
            return ((phi + 15) & ~size_t(15)) + (split ? rec : 0) +
                   (size_t)2 * kXchDirs * (kTX + 2) * TY * real_size(p) + (size_t)2 * 3 * TY * 2 * real_size(p);
    }
}

// Tile rows: preferred per kind and storage (measured on MI355X), else the
// largest that keeps the LDS rings within the per-workgroup budget.
int tile_rows(const lb_params& p, int kind) {
    if (kind == TILE_SINGLE) {
        // FP32 lattices of 2^23 sites or more take 16 rows (1024-thread
        // workgroups, one per CU: the autotuner's choice at 256^3) when they
        // split into whole rounds of 256 such workgroups, so that no CU idles
        // (measured: 384^3 with 144 of them ran 24 % slower than with 8 rows);
        // other lattices take 8 (16-bit storage too: with its record ring that
        // is one workgroup of 8 waves per CU, measured faster than two
        // workgroups of 4 rows)
        const int set = tile_setting(TILE_SINGLE, p.storage).ty;
        int dflt = kSingleTY;
        if (p.storage == LB_STORE_F32 && set <= 0 && (size_t)p.nx * p.ny * p.nz >= ((size_t)1 << 23)) {
            const int tiles = ((p.nx + kTX - 1) / kTX) * ((p.ny + kSingleTYLarge - 1) / kSingleTYLarge);
            const int want_chunks = std::max(1, 256 / tiles);
            const int tz = std::max(4 * tile_halo(p), (p.nz + want_chunks - 1) / want_chunks);
            const int blocks = tiles * ((p.nz + tz - 1) / tz);
            if (blocks % 256 == 0) dflt = kSingleTYLarge;
        }
        const int want = set > 0 ? set : env_int("LB_SINGLE_TY", dflt);
        for (int ty : {want, kSingleTY, kSingleTYSmall})
            if ((ty == kSingleTY || ty == kSingleTYSmall || ty == kSingleTYLarge) &&
                tile_lds(p, kind, ty) <= (size_t)device_lds_bytes())
                return ty;
        return 0;
    }
    const char* env = kind == TILE_PHASE ? "LB_PHASE_TY" : "LB_COLLIDE_TY";
    int want = tile_setting(kind, p.storage).ty;
    if (want <= 0) want = env_int(env, 0);
    if (want <= 0) {
        // the autotuner's choices for the 256^3 emulsion on MI355X
        if (kind == TILE_PHASE) want = 4;
        else if (split_storage(p)) want = kind == TILE_COLLIDE ? 4 : 8;
        else want = p.storage == LB_STORE_F64 ? 8 : 4;
    }
    for (int ty = want; ty >= 1; ty /= 2)
        if (tile_lds(p, kind, ty) <= (size_t)max_lds_bytes()) return ty;
    return 0;
}

FusedShape tile_shape(const lb_params& p, int kind, int target_blocks) {
    FusedShape fs;
    fs.TY = tile_rows(p, kind);
    fs.tiles_x = (p.nx + kTX - 1) / kTX;
    fs.tiles_y = (p.ny + fs.TY - 1) / fs.TY;
    const int tiles = fs.tiles_x * fs.tiles_y;
    int tz = tile_setting(kind, p.storage).tz;
    if (tz <= 0) tz = env_int(kind == TILE_PHASE ? "LB_PHASE_TZ" : "LB_TZ", 0);
    // the autotuner's choices for the 256^3 emulsion on MI355X: 16-plane chunks
    // for the 16-bit phase pass and the raw-storage two-pass collide
    if (tz <= 0 && (kind == TILE_PHASE || (kind == TILE_COLLIDE && !split_storage(p)))) tz = 16;
    // one-read tiles that fill a CU alone -- 16-row tiles (1024 threads) and
    // 16-bit storage's 8-row tiles (their LDS rings) -- aim for one round of
    // 256 workgroups (deep chunks: fewer halo planes and face sites; measured
    // at 256^3: fp16 1.31 ms/step with 32-plane chunks, 1.23 ms with 128)
    if (kind == TILE_SINGLE && (fs.TY == kSingleTYLarge || (split_storage(p) && fs.TY == kSingleTY)))
        target_blocks = 256;
    if (tz <= 0) {
        // aim for target_blocks workgroups, keeping chunks a few halos deep
        const int H = kind == TILE_PHASE ? 1 : tile_halo(p);
        const int want_chunks = std::max(1, target_blocks / std::max(1, tiles));
        tz = std::max(4 * H, (p.nz + want_chunks - 1) / want_chunks);
    }
    fs.TZ = std::min(std::max(tz, 1), p.nz);
    fs.chunks = (p.nz + fs.TZ - 1) / fs.TZ;
    fs.nblocks = tiles * fs.chunks;
    return fs;
}

int choose_kernel(const lb_params& p) {
    const bool fits = tile_rows(p, TILE_SINGLE) > 0;
    if (p.kernel == LB_KERNEL_TWOPASS) return LB_KERNEL_TWOPASS;
    if (p.kernel == LB_KERNEL_FUSED) return fits ? LB_KERNEL_FUSED : -1;
    // automatic: the one-read step (measured faster than two passes for raw
    // and 16-bit storage); the Shan-Chen model and lattices too large for
    // 32-bit buffer offsets take two passes
    // (the one-read step's 32-bit byte offsets need 10 x raw_stride(sites) x value size < 2^32)
    const bool small =
        (uint64_t)kResArrays * real_size(p) * (uint64_t)raw_stride((size_t)p.nx * p.ny * p.nz) < ((uint64_t)1 << 32);
    if (!fits || !small || p.model != LB_MODEL_COLOUR_GRADIENT) return LB_KERNEL_TWOPASS;
    return LB_KERNEL_FUSED;
}

// Source/destination storage pairs a step may combine: same storage, or the
// raw FP32 initial state of a 16-bit lattice into its moment-split storage.
template <typename Src, typename Dst>
struct StepPair : std::false_type {};
template <typename T, bool MW>
struct StepPair<RawPop<T, MW>, RawPop<T>> : std::true_type {};
template <typename H>
struct StepPair<RawPop<float>, SplitPop<H>> : std::true_type {};
template <typename H, bool MW>
struct StepPair<SplitPop<H, MW>, SplitPop<H>> : std::true_type {};

template <typename Dst>
int step_into(const LatticeView& v, int kernel, const Dst& dst, const StepEvents* t) {
    return with_state(v, [&](auto rt, auto src, const auto& c) {
        using R = decltype(rt);
        using S = decltype(src);
        if constexpr (StepPair<S, Dst>::value) return step_with<R>(v, kernel, src, dst, c, t);
        return set_error(LB_EINVAL, "storage/compute mismatch");
    });
}

int launch_step(const LatticeView& v, int kernel, const StepEvents* t) {
    const size_t N = (size_t)v.g.N;
    switch (v.p->storage) {
        case LB_STORE_F64: return step_into(v, kernel, RawPop<double>{(double*)v.nxt, N}, t);
        case LB_STORE_F32: return step_into(v, kernel, RawPop<float>{(float*)v.nxt, N}, t);
        case LB_STORE_F16: return step_into(v, kernel, split_view<__half>(v.nxt, N, v.p->scale_log2), t);
        case LB_STORE_BF16: return step_into(v, kernel, split_view<__hip_bfloat16>(v.nxt, N, v.p->scale_log2), t);
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

int launch_korteweg(const LatticeView& v, double lam, int b, void* kout, void* pout, int dtype, int accumulate) {
    return with_state(v, [&](auto rt, auto src, const auto&) {
        using R = decltype(rt);
        using S = decltype(src);
        // phase field of the current state, as the next collision sees it: a
        // one-read state completes the field its phase-sum buffer holds (the
        // next step repeats that, with the same result); otherwise a phase
        // pass writes it into the scratch field
        const R* field = (const R*)v.phi;
        int rc;
        if (v.part_valid && v.part_in) {
            const FusedShape fs = tile_shape(*v.p, TILE_SINGLE);
            if (fs.TY == kSingleTY) rc = assemble_phase<R, S, kSingleTY>(v, src, fs);
            else if (fs.TY == kSingleTYLarge) rc = assemble_phase<R, S, kSingleTYLarge>(v, src, fs);
            else rc = assemble_phase<R, S, kSingleTYSmall>(v, src, fs);
            field = phi_of<kTX>((Part2<R>*)v.part_in, v.g);
        } else {
            rc = phase_pass<R>(v, src);
        }
        if (rc) return rc;
        const dim3 grid((unsigned)(((v.g.nx + 63) / 64) * ((v.g.ny + kKortewegRows - 1) / kKortewegRows) *
                                   ((v.g.nz + kKortewegChunk - 1) / kKortewegChunk)));
        const dim3 block(64 * kKortewegRows);
        if (dtype == LB_DTYPE_F64)
            hipLaunchKernelGGL((korteweg_kernel<R, double>), grid, block, 0, v.stream, v.g, field, R(lam),
                               b, (double*)kout, (double*)pout, accumulate);
        else
            hipLaunchKernelGGL((korteweg_kernel<R, float>), grid, block, 0, v.stream, v.g, field, R(lam),
                               b, (float*)kout, (float*)pout, accumulate);
        return launch_status("korteweg_kernel");
    });
}

int launch_droplets(hipStream_t st, const Geom& g, const double* cen, const double* rad, int n, double width,
                    double background, double rho0, double* rr, double* rb) {
    hipLaunchKernelGGL(droplet_fields_kernel, dim3(grid_for(g.N)), dim3(kBlock), 0, st, g, cen, rad, n, width,
                       background, rho0, rr, rb);
    return launch_status("droplet_fields_kernel");
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
