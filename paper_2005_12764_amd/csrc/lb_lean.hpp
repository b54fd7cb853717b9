// lb_lean.hpp -- the one-read step for raw (FP64/FP32) storage, written for
// the CDNA4 instruction mix.
//
// Same step and same phase-sum bookkeeping as single_tile (lb_single.hpp):
// the tile collides and streams its sites and gathers, in the same fixed
// order, the own phase sums of the next state.  What differs is how the work
// maps onto a wavefront:
//   - a tile row is one wavefront, so the row's y and the plane's z are
//     wave-uniform: every upstream row offset (periodic wrap, wall tests) is
//     scalar arithmetic, and each of the 38 pulls and 38 stores is a global
//     access with a scalar row base plus one of three loop-invariant per-lane
//     column offsets (x, x-1, x+1 with the periodic wrap);
//   - the phase-field ring is staged row by row with scalar row addresses;
//   - neighbours in the same row are read with DPP wavefront shifts that fill
//     the lane beyond the row's end with zero, so a source outside the tile
//     (or beyond an x wall) contributes nothing without a per-lane test, and
//     the shift folds into the add that consumes it;
//   - values for other rows go through LDS rows padded with a zero at both
//     ends, for the same reason;
//   - every lane runs the collision (lanes beyond the lattice on clamped
//     coordinates); only stores are masked.
// The kernel the step launched before (single_kernel) computes the same
// quantities; the two agree to rounding (the collision is shared).
#pragma once
#include "lb_single.hpp"

namespace lbm {

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
// Keep a wave-uniform value in a vector register.
__device__ __forceinline__ void in_vgpr(float& v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void in_vgpr(double& v) { asm volatile("" : "+v"(v)); }

// The 19 (t_i, d_i) pair arrays of a raw buffer as four buffer resources of
// up to five arrays (ten values per site) each: a pull or store is then one
// buffer access of a pair with the row in a scalar offset and the column in a
// per-lane offset, with no 64-bit address arithmetic per access.  Each range
// is exact, so an access outside it reads zero or is dropped.  Needs
// 10 raw_stride(N) sizeof(T) < 2^32 (checked on the host).
constexpr int kResArrays = 10;
constexpr int kResPairs = kResArrays / 2;
constexpr unsigned kRsrcWord3 = 0x00020000;  // raw 32-bit buffer on gfx9-family targets
template <typename T>
struct PopRes {
    __amdgpu_buffer_rsrc_t r[4];
    // S: pairs from one array to the next (raw_stride(N))
    __device__ __forceinline__ PopRes(const T* f, unsigned S) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const unsigned np = (unsigned)min(kResPairs, Q - k * kResPairs);
            r[k] = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(f) + (size_t)k * kResArrays * S, 0,
                                                     (int)(np * S * 2u * (unsigned)sizeof(T)), (int)kRsrcWord3);
        }
    }
};
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
// (t, d) pair loads and non-temporal pair stores
__device__ __forceinline__ void res_load_pair(float& t, float& d, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                              unsigned soff) {
    const auto v = __builtin_bit_cast(RawPair<float>::type, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    t = v.x;
    d = v.y;
}
__device__ __forceinline__ void res_load_pair(double& t, double& d, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                              unsigned soff) {
    const auto v = __builtin_bit_cast(RawPair<double>::type, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    t = v.x;
    d = v.y;
}
__device__ __forceinline__ void res_store_pair(float t, float d, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                               unsigned soff) {
    RawPair<float>::type v;
    v.x = t;
    v.y = d;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 2);
}
__device__ __forceinline__ void res_store_pair(double t, double d, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                               unsigned soff) {
    RawPair<double>::type v;
    v.x = t;
    v.y = d;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, voff, soff, 2);
}
__device__ __forceinline__ float res_load(float, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ double res_load(double, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
// non-temporal store (aux = 2: nt)
__device__ __forceinline__ void res_store(float v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 2);
}
__device__ __forceinline__ void res_store(double v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, voff, soff, 2);
}

// Resource over n values of an array whose pointer is made opaque first (the
// resource is then rebuilt where it is used instead of held in scalar
// registers across the loop).
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t array_res(const T* p, unsigned n) {
    asm volatile("" : "+s"(p));
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p), 0, (int)(n * (unsigned)sizeof(T)), (int)kRsrcWord3);
}
// phase-sum pair (own sums of a face site), 8 or 16 bytes
__device__ __forceinline__ void res_store(const Part2<float>& v, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                          unsigned soff) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, voff, soff, 0);
}
__device__ __forceinline__ void res_store(const Part2<double>& v, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                          unsigned soff) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V, v), r, voff, soff, 0);
}
__device__ __forceinline__ void res_store_cached(float v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}
__device__ __forceinline__ void res_store_cached(double v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, voff, soff, 0);
}

// Value of lane l-1 of the wavefront (0 in lane 0) and of lane l+1 (0 in
// lane 63): DPP wave_shr:1 / wave_shl:1 with out-of-range lanes reading zero.
__device__ __forceinline__ float from_left(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_right(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double from_left(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double from_right(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Upstream row (scalar): element offset (z*ny + y)*nx of the row a population
// with velocity (., cy, cz) arriving in row (y, z) comes from, with the
// periodic wrap.  W: the lattice may have walls; `bb` is then set when that
// row lies beyond one (the population is a bounce-back).
template <bool W>
__device__ __forceinline__ unsigned upstream_row(const Geom& g, int y, int z, int cy, int cz, bool& bb) {
    int ys = y - cy, zs = z - cz;
    const bool out_y = ys < 0 || ys >= g.ny, out_z = zs < 0 || zs >= g.nz;
    ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
    zs = zs < 0 ? zs + g.nz : (zs >= g.nz ? zs - g.nz : zs);
    bb = W && ((g.wy && out_y) || (g.wz && out_z));
    return (unsigned)((zs * g.ny + ys) * g.nx);
}

// Plane and lane context of the pulls and stores of a lean tile.
struct LeanPlane {
    unsigned Np;       // sites N, re-read each plane (keeps array offsets out of loop-invariant registers)
    unsigned own_row;  // (cz ny + yc) nx, the site's row
    int yc, cz;        // the site's (clamped) row and its plane
    int rs[3];         // record-ring slots of planes cz - 1, cz, cz + 1 (16-bit storage)
};
struct LeanLane {
    unsigned cx0, cxm, cxp;   // columns x, x - 1, x + 1 (periodic wrap; beyond an x wall x itself)
    bool wall_xlo, wall_xhi;  // an x wall lies beyond this lane's site
    int lane, ty;
};

// Raw storage: (t_i, d_i) pairs in Q arrays.  Pulls read each array at the
// upstream row (scalar offset) and column (per lane); stores write in place.
// The pulls load their values where they need them: loading them one plane
// ahead takes 2 Q more vector registers, and the occupancy that costs (FP32:
// 4 -> 2 waves per SIMD) measured slower (256^3: 1.30 against 1.12 ms).
template <typename T>
struct LeanRaw {
    using R = T;
    static constexpr bool split = false;
    const T* fin;
    T* fout;
    __host__ __device__ static constexpr size_t ring_bytes(int) { return 0; }
    struct Pre {};
    __device__ __forceinline__ void stage_load(const Geom&, int, int, int, int, int, Pre&) const {}
    __device__ __forceinline__ void stage_store(int, int, int, const Pre&) const {}

    // t_i, d_i of site (x, yc, cz): direction i at the upstream site, or (a
    // bounce-back off a y or z wall) the opposite direction at the site itself
    template <bool W>
    __device__ __forceinline__ void load(const Geom& g, int yc, int cz, const LeanLane& ln, T (&t)[Q],
                                         T (&d)[Q]) const {
        using L = Lattice;
        unsigned Sp = (unsigned)raw_stride((size_t)g.N);
        asm volatile("" : "+s"(Sp));
        const T* fin_p = fin;
        asm volatile("" : "+s"(fin_p));  // resources rebuilt each plane (short-lived scalar registers)
        const PopRes<T> fi(fin_p, Sp);
        constexpr unsigned SZ = 2 * (unsigned)sizeof(T);  // bytes of a (t, d) pair
        const unsigned bx0 = ln.cx0 * SZ, bxm = ln.cxm * SZ, bxp = ln.cxp * SZ;
        const unsigned own_row = (unsigned)((cz * g.ny + yc) * g.nx);
        // byte offset of direction i's pair at site e within its resource
        auto soff = [&](int i, unsigned e) { return ((unsigned)(i % kResPairs) * Sp + e) * SZ; };
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            bool bb;
            const unsigned row = upstream_row<W>(g, yc, cz, L::cy[i], L::cz[i], bb);
            const unsigned col = L::cx[i] > 0 ? bxm : (L::cx[i] < 0 ? bxp : bx0);
            if (W && bb) {
                const int o = L::opp[i];
                res_load_pair(t[i], d[i], fi.r[o / kResPairs], bx0, soff(o, own_row));
            } else {
                res_load_pair(t[i], d[i], fi.r[i / kResPairs], col, soff(i, row));
            }
        }
    }
    template <bool W>
    __device__ __forceinline__ void dev_load(const Geom&, int, int, const LeanLane&, Pre&) const {}

    // MV: the lattice may have moving walls (resting-wall kernels carry none
    // of that code)
    template <bool W, bool MV>
    __device__ __forceinline__ void pull(const Geom& g, const LeanPlane& P, const LeanLane& ln, const Pre&,
                                         R (&t)[Q], R (&d)[Q]) const {
        using L = Lattice;
        load<W>(g, P.yc, P.cz, ln, t, d);
        if constexpr (W) {
            // lanes next to an x wall: their bounce-backs, from the site itself
            constexpr unsigned SZ = 2 * (unsigned)sizeof(T);
            const unsigned bx0 = ln.cx0 * SZ;
            const unsigned Sp = P.Np + kRawPad;
            auto soff = [&](int i, unsigned e) { return ((unsigned)(i % kResPairs) * Sp + e) * SZ; };
            const T* fin_p = fin;
            asm volatile("" : "+s"(fin_p));
            const PopRes<T> fi(fin_p, Sp);
            if (ln.wall_xlo || ln.wall_xhi) {
#pragma unroll
                for (int i = 1; i < Q; ++i) {
                    if (!((L::cx[i] > 0 && ln.wall_xlo) || (L::cx[i] < 0 && ln.wall_xhi))) continue;
                    const int o = L::opp[i];
                    res_load_pair(t[i], d[i], fi.r[o / kResPairs], bx0, soff(o, P.own_row));
                }
            }
            // moving walls: each reflected direction gains the wall term,
            // shared between the components by the site's own post-collision
            // phase (as RawPop::add_wall_terms)
            const bool wyz = (g.wy && (P.yc == 0 || P.yc == g.ny - 1)) || (g.wz && (P.cz == 0 || P.cz == g.nz - 1));
            if (MV && g.moving && (wyz || ln.wall_xlo || ln.wall_xhi)) {
                R st = R(0), sd = R(0);
                for (int j = 0; j < Q; ++j) {
                    R tj, dj;
                    res_load_pair(tj, dj, fi.r[j / kResPairs], bx0, soff(j, P.own_row));
                    st += weight<R>(j) + tj;
                    sd += dj;
                }
                const R ph = sd / st;
#pragma unroll
                for (int i = 1; i < Q; ++i) {
                    bool bb;
                    (void)upstream_row<W>(g, P.yc, P.cz, L::cy[i], L::cz[i], bb);
                    const bool rx = (L::cx[i] > 0 && ln.wall_xlo) || (L::cx[i] < 0 && ln.wall_xhi);
                    if (!(bb || rx)) continue;
                    const R add = wall_term<R>(g, i, (int)ln.cx0, P.yc, P.cz);
                    t[i] += add;
                    d[i] += add * ph;
                }
            }
        }
    }

    // Store, and keep in t, d the values a later pull reads.
    __device__ __forceinline__ void store(const Geom&, const LeanPlane& P, const LeanLane& ln, R (&t)[Q],
                                          R (&d)[Q], const SiteTotals<R>&, bool site_in) const {
        if (site_in) {
            T* fout_p = fout;
            asm volatile("" : "+s"(fout_p));
            const unsigned Sp = P.Np + kRawPad;
            const PopRes<T> fo(fout_p, Sp);
            constexpr unsigned SZ = 2 * (unsigned)sizeof(T);
            auto soff = [&](int i, unsigned e) { return ((unsigned)(i % kResPairs) * Sp + e) * SZ; };
#pragma unroll
            for (int i = 0; i < Q; ++i) res_store_pair(T(t[i]), T(d[i]), fo.r[i / kResPairs], ln.cx0 * SZ, soff(i, P.own_row));
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            t[i] = R(T(t[i]));
            d[i] = R(T(d[i]));
        }
    }
};

// 16-bit moment-split storage (the codec of SplitPop): per site an FP32
// record of 8 values, per direction a 16-bit deviation.  The records of
// planes cz - 1, cz, cz + 1 (tile plus one site) sit in an LDS ring, staged a
// plane ahead, so a pull reads its source record from LDS and only the 16-bit
// deviation from memory (scalar row offset, per-lane column).
__device__ __forceinline__ f4 res_load4(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
__device__ __forceinline__ void res_store4(f4 v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V, v), r, voff, soff, 2);
}
template <typename H>
struct LeanSplit {
    using R = float;
    static constexpr bool split = true;
    static constexpr int LXR = kTX + 2;  // ring row: the tile's 64 columns and one on each side
    const float* rin;                   // records [N][8] of the current state
    const H* din;                       // deviations [Q][N] of the current state
    float* rout;                        // the same of the next state
    H* dout;
    SplitPop<H> codec;                  // scale and the record arithmetic
    f4* ring;                           // LDS: 3 planes x 2 halves x (TY + 2) rows x LXR sites, f4
    int TY;
    __host__ __device__ static constexpr size_t ring_bytes(int ty) {
        return (size_t)3 * (ty + 2) * LXR * 2 * sizeof(f4);
    }
    // a plane holds the first f4 of every site, then (half() later) the second:
    // consecutive lanes read consecutive 16-byte words, free of bank conflicts
    __device__ __forceinline__ f4* plane(int slot) const { return ring + (size_t)slot * (TY + 2) * LXR * 2; }
    __device__ __forceinline__ int half() const { return (TY + 2) * LXR; }
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t rec_res(const float* p, unsigned N) const {
        asm volatile("" : "+s"(p));
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), 0, (int)(N * 32u), (int)kRsrcWord3);
    }
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t dev_res(const H* p, unsigned N) const {
        asm volatile("" : "+s"(p));
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<H*>(p), 0, (int)(Q * (N + kDevPad) * 2u), (int)kRsrcWord3);
    }

    // Loaded one plane ahead, so that their latency overlaps a collision:
    // records of two ring rows (and of the two columns past the tile) for the
    // next staging, and the 16-bit deviations of the next site's pulls.
    struct Pre {
        f4 a0[2], a1[2], b0[2], b1[2];
        unsigned dv[Q];  // the 16-bit deviations, one per register (two per register would make
                         // every load wait at once for the packing)
    };
    static __device__ __forceinline__ H dev_of(unsigned v) { return __builtin_bit_cast(H, (unsigned short)v); }

    // Records of plane q, rows y0 - 1 .. y0 + TY and columns x0 - 1 .. x0 + 64
    // (periodic wrap or mirror images beyond walls): loaded into registers,
    // then (stage_store) written to a ring slot.  Thread row ty takes ring
    // rows ty and ty + TY (TY >= 2: at most two rows).
    __device__ __forceinline__ void stage_load(const Geom& g, int q, int x0, int y0, int ty, int lane,
                                               Pre& pr) const {
        const int zz = halo_coord(q, g.nz, g.wz);
        const unsigned ca = (unsigned)halo_coord(x0 - 1 + lane, g.nx, g.wx) * 32u;
        const unsigned cb = (unsigned)halo_coord(x0 - 1 + kTX + lane, g.nx, g.wx) * 32u;
        const __amdgpu_buffer_rsrc_t rr = rec_res(rin, (unsigned)g.N);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int r = ty + k * TY;
            if (r < TY + 2) {
                const int yy = halo_coord(y0 - 1 + r, g.ny, g.wy);
                const unsigned so = (unsigned)((zz * g.ny + yy) * g.nx) * 32u;
                pr.a0[k] = res_load4(rr, ca, so);
                pr.a1[k] = res_load4(rr, ca + 16u, so);
                if (lane < 2) {
                    pr.b0[k] = res_load4(rr, cb, so);
                    pr.b1[k] = res_load4(rr, cb + 16u, so);
                }
            }
        }
    }
    __device__ __forceinline__ void stage_store(int slot, int ty, int lane, const Pre& pr) const {
        f4* pl = plane(slot);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int r = ty + k * TY;
            if (r < TY + 2) {
                pl[r * LXR + lane] = pr.a0[k];
                pl[half() + r * LXR + lane] = pr.a1[k];
                if (lane < 2) {
                    pl[r * LXR + kTX + lane] = pr.b0[k];
                    pl[half() + r * LXR + kTX + lane] = pr.b1[k];
                }
            }
        }
    }

    // Deviations the pulls of site (x, yc, cz) read: direction i at the
    // upstream site, or (a bounce-back off a y or z wall) the opposite
    // direction at the site itself; the lanes next to an x wall re-read
    // theirs in pull.
    template <bool W>
    __device__ __forceinline__ void dev_load(const Geom& g, int yc, int cz, const LeanLane& ln, Pre& pr) const {
        using L = Lattice;
        unsigned Np = (unsigned)g.N;
        asm volatile("" : "+s"(Np));
        const unsigned own_row = (unsigned)((cz * g.ny + yc) * g.nx);
        const __amdgpu_buffer_rsrc_t dr = dev_res(din, Np);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            bool bb;
            const unsigned row = upstream_row<W>(g, yc, cz, L::cy[i], L::cz[i], bb);
            const int a = (W && bb) ? L::opp[i] : i;
            const unsigned col = (W && bb) ? ln.cx0 : (L::cx[i] > 0 ? ln.cxm : (L::cx[i] < 0 ? ln.cxp : ln.cx0));
            const unsigned rw = (W && bb) ? own_row : row;
            pr.dv[i] = __builtin_amdgcn_raw_buffer_load_b16(dr, col * 2u, ((unsigned)a * (Np + kDevPad) + rw) * 2u, 0);
        }
    }

    template <bool W, bool MV>
    __device__ __forceinline__ void pull(const Geom& g, const LeanPlane& P, const LeanLane& ln, const Pre& pr,
                                         R (&t)[Q], R (&d)[Q]) const {
        using L = Lattice;
        const f4* pm = plane(P.rs[0]);
        const f4* p0 = plane(P.rs[1]);
        const f4* pp = plane(P.rs[2]);
        const int own = (ln.ty + 1) * LXR + ln.lane + 1;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            bool bb;
            (void)upstream_row<W>(g, P.yc, P.cz, L::cy[i], L::cz[i], bb);
            if (W && bb) {
                codec.decode(i, L::opp[i], p0[own], p0[half() + own], dev_of(pr.dv[i]), t[i], d[i]);
            } else {
                // the source (x - c_i) in plane cz - c_z: cz - 1 is pm, cz + 1 is pp
                const f4* pl = L::cz[i] > 0 ? pm : (L::cz[i] < 0 ? pp : p0);
                const int pos = own - L::cy[i] * LXR - L::cx[i];
                codec.decode(i, i, pl[pos], pl[half() + pos], dev_of(pr.dv[i]), t[i], d[i]);
            }
        }
        if constexpr (W) {
            if (ln.wall_xlo || ln.wall_xhi) {
                const __amdgpu_buffer_rsrc_t dr = dev_res(din, P.Np);
#pragma unroll
                for (int i = 1; i < Q; ++i) {
                    if (!((L::cx[i] > 0 && ln.wall_xlo) || (L::cx[i] < 0 && ln.wall_xhi))) continue;
                    const int o = L::opp[i];
                    const H dv = __builtin_bit_cast(H, __builtin_amdgcn_raw_buffer_load_b16(
                                                           dr, ln.cx0 * 2u, ((unsigned)o * (P.Np + kDevPad) + P.own_row) * 2u, 0));
                    codec.decode(i, o, p0[own], p0[half() + own], dv, t[i], d[i]);
                }
            }
            // moving walls: each reflected direction gains the wall term,
            // shared by the phase of the site's own record (as
            // SplitPop::add_wall_terms)
            const bool wyz = (g.wy && (P.yc == 0 || P.yc == g.ny - 1)) || (g.wz && (P.cz == 0 || P.cz == g.nz - 1));
            if (MV && g.moving && (wyz || ln.wall_xlo || ln.wall_xhi)) {
                const float ph = p0[half() + own].x;
#pragma unroll
                for (int i = 1; i < Q; ++i) {
                    bool bb;
                    (void)upstream_row<W>(g, P.yc, P.cz, L::cy[i], L::cz[i], bb);
                    const bool rx = (L::cx[i] > 0 && ln.wall_xlo) || (L::cx[i] < 0 && ln.wall_xhi);
                    if (!(bb || rx)) continue;
                    const R add = wall_term<R>(g, i, (int)ln.cx0, P.yc, P.cz);
                    t[i] += add;
                    d[i] += add * R(ph);
                }
            }
        }
    }

    // Encode and store the record and the deviations, and keep in t, d the
    // values a later pull decodes (exactly: the same codec arithmetic).
    __device__ __forceinline__ void store(const Geom& g, const LeanPlane& P, const LeanLane& ln, R (&t)[Q],
                                          R (&d)[Q], const SiteTotals<R>& tot, bool site_in) const {
        const f4 ra = {tot.drho, tot.jx, tot.jy, tot.jz};
        const f4 rb = {tot.phi, tot.vx, tot.vy, tot.vz};
        H h[Q];
        float X[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            X[i] = SplitPop<H>::excess(i, 1.0f, ra);
            h[i] = Half<H>::from_f((t[i] - weight<float>(i) * X[i]) * codec.scale);
        }
        if (site_in) {
            const __amdgpu_buffer_rsrc_t rr = rec_res(rout, P.Np);
            const __amdgpu_buffer_rsrc_t dr = dev_res(dout, P.Np);
            res_store4(ra, rr, ln.cx0 * 32u, P.own_row * 32u);
            res_store4(rb, rr, ln.cx0 * 32u + 16u, P.own_row * 32u);
#pragma unroll
            for (int i = 0; i < Q; ++i)
                __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, h[i]), dr, ln.cx0 * 2u,
                                                      ((unsigned)i * (P.Np + kDevPad) + P.own_row) * 2u, 2);
        }
        (void)g;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            float tt, dd;
            codec.finish(i, 1.0f, X[i], rb, h[i], tt, dd);
            t[i] = tt;
            d[i] = dd;
        }
    }
};

// Exchange rows in LDS: per tile row, kXchDirs x 2 values (w_i + t_i, d_i)
// of the directions with c_y != 0, each a row of 64 lanes with a zero pad
// before and after it.
constexpr int kLeanRowPad = kTX + 2;
template <typename R, int TY>
__host__ __device__ constexpr size_t lean_xch_bytes() {
    return (size_t)TY * 2 * kXchDirs * kLeanRowPad * sizeof(R);
}

// As xedge_rows, reading the exchange rows of the lean tile: the in-plane
// terms from the rows above and below that the edge lanes of those rows send
// across this x face (ascending direction); the chunk's last plane is then
// complete.
template <typename R, int TY, int SX>
__device__ __forceinline__ void lean_xedge_rows(const Geom& g, const R* __restrict__ xch, Part2<R>* __restrict__ vs,
                                                int ty, int tx, int nrows, int y, int cz, int za, int zb, int bd,
                                                Part2<R>* __restrict__ xf) {
    using L = Lattice;
    constexpr int XROW = 2 * kXchDirs * kLeanRowPad;
    constexpr int side = SX < 0 ? 0 : 1;
    Part2<R>* v = vs + side * 3 * TY + ty;
    Part2<R> P = v[((cz - za) % 3) * TY];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (L::cx[i] != SX || L::cz[i] != 0 || L::cy[i] == 0) continue;
        const int ys = ty - L::cy[i];
        if (ys < 0 || ys >= nrows) continue;
        const R* src = xch + ys * XROW + 1 + tx;
        P.rc += src[(2 * xch_slot(i)) * kLeanRowPad];
        P.dn += src[(2 * xch_slot(i) + 1) * kLeanRowPad];
    }
    if (cz == zb - 1) xf[xface_at(g, bd, 1 - side, y, cz)] = P;
    else v[((cz - za) % 3) * TY] = P;
}

// One tile of the lean one-read step: columns [x0, x0+64) x [y0, y0+TY),
// planes [za, zb); blockDim.x == 64 * TY.  W: the lattice has walls (an
// all-periodic lattice carries none of their tests; the lanes next to an x
// wall take their bounce-backs from a second, masked pull).
template <typename S, int TY, int H, bool W, bool MV = false>
__device__ __forceinline__ void lean_tile(const Geom& g, const S& st, const Coeffs<typename S::R>& cs,
                                          typename S::R* __restrict__ ringb, typename S::R* __restrict__ xch,
                                          Part2<typename S::R>* __restrict__ vs, int x0, int y0, int za, int zb,
                                          const typename S::R* __restrict__ phi_in,
                                          Part2<typename S::R>* __restrict__ part_out,
                                          typename S::R* __restrict__ phi_out, int moving_next) {
    using L = Lattice;
    using R = typename S::R;
    constexpr int TX = kTX;
    constexpr int LX = TX + 2 * H;
    constexpr int NP = 2 * H + 1;
    constexpr int LY = TY + 2 * H;
    constexpr int PLANE = LY * LX;
    constexpr int XROW = 2 * kXchDirs * kLeanRowPad;  // exchange reals per tile row
    const unsigned N = (unsigned)g.N;  // byte offsets within a resource < 2^32 (checked on the host)
    // the collision's real coefficients in vector registers: the loop holds
    // more wave-uniform values than the scalar register file, and a VALU
    // operation reads a vector register at no cost (the flags that steer
    // control flow stay scalar)
    Coeffs<R> c = cs;
    in_vgpr(c.inv_nu_r);
    in_vgpr(c.inv_nu_b);
    in_vgpr(c.omega);
    in_vgpr(c.half_A);
    in_vgpr(c.beta);
    in_vgpr(c.eps_g);
    in_vgpr(c.eps_g2);
    in_vgpr(c.g_iface);
    in_vgpr(c.g_iface2);
    in_vgpr(c.nc_strength);
    in_vgpr(c.nc_hmin);
    in_vgpr(c.fx);
    in_vgpr(c.fy);
    in_vgpr(c.fz);
    const int lane = threadIdx.x & 63;
    const int ty = wave_uniform(threadIdx.x >> 6);
    const int x = x0 + lane;
    const int y = y0 + ty;
    const int x1 = min(x0 + TX, g.nx), y1 = min(y0 + TY, g.ny);
    const int nrows = y1 - y0;
    const bool xin = x < g.nx;
    const bool row_in = y < g.ny;
    const bool ragged = x1 - x0 < TX;
    // clamped coordinates: lanes and rows beyond the lattice compute on a
    // valid site and store nothing
    const int xc = xin ? x : g.nx - 1;
    const int yc = row_in ? y : g.ny - 1;
    // per-lane column offsets of the pulls: x, x - 1 and x + 1 with the wrap
    // (beyond an x wall the lane's own column; its bounce-back is re-pulled)
    const unsigned cx0 = (unsigned)xc;
    const bool WX = W && g.wx;
    const unsigned cxm = (unsigned)(xc == 0 ? (WX ? 0 : g.nx - 1) : xc - 1);
    const unsigned cxp = (unsigned)(xc == g.nx - 1 ? (WX ? xc : 0) : xc + 1);
    const bool wall_xlo = WX && xc == 0, wall_xhi = WX && xc == g.nx - 1;
    const LeanLane ln{cx0, cxm, cxp, wall_xlo, wall_xhi, lane, ty};
    // phase-ring columns of this lane: x0 - H + lane and x0 - H + 64 + lane
    const int ra = halo_coord(x0 - H + lane, g.nx, g.wx);
    const int rb = halo_coord(x0 - H + TX + lane, g.nx, g.wx);
    // edge lanes of the row and the columns their x-face sums go to
    Part2<R>* const xf = part_out + g.N;
    int bd_lo = 0, bd_hi = 0;
    const bool edge_lo = row_in && lane == 0 && xface_dest<TX>(g, x0, x1, -1, bd_lo);
    const bool edge_hi = row_in && x == x1 - 1 && xface_dest<TX>(g, x0, x1, 1, bd_hi);
    // zero pads of this row's exchange slots
    R* const xrow = xch + ty * XROW;
    if (lane < 2 * kXchDirs) {
        xrow[lane * kLeanRowPad] = R(0);
        xrow[lane * kLeanRowPad + kLeanRowPad - 1] = R(0);
    }
    R prev_dn = R(0), prev_rc = R(0), cur_dn = R(0), cur_rc = R(0);

    // phase field of plane q on the tile and its halo, rows ty, ty + TY, ...:
    // loaded into registers one plane ahead, so that the loads of plane p + 1
    // are in flight while plane p is collided
    constexpr int NR = (LY + TY - 1) / TY;
    R pfa[NR], pfb[NR];
    auto fetch = [&](int q) {
        const int zz = halo_coord(q, g.nz, g.wz);
        const __amdgpu_buffer_rsrc_t pr = array_res(phi_in, N);
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int r = ty + k * TY;
            if (r < LY) {
                const int yy = halo_coord(y0 - H + r, g.ny, g.wy);
                const unsigned so = (unsigned)((zz * g.ny + yy) * g.nx) * (unsigned)sizeof(R);
                pfa[k] = res_load(R(0), pr, (unsigned)ra * (unsigned)sizeof(R), so);
                pfb[k] = lane < 2 * H ? res_load(R(0), pr, (unsigned)rb * (unsigned)sizeof(R), so) : R(0);
            }
        }
    };
    fetch(za - H);
    // Values loaded one plane ahead (records to stage, deviations to pull)
    // are loaded in every iteration, at the same point, for a plane clamped
    // into the lattice: a value the loop carries then has a single source,
    // and no register copy at the loop head has to wait for its load.  The
    // loads of planes nothing uses are in bounds and few.
    typename S::Pre pre;
    st.stage_load(g, za - 2 * H + 1, x0, y0, ty, lane, pre);

    for (int p = za - H; p < zb + H; ++p) {
        const int slot = (p - (za - H)) % NP;
        // ---- phase field of plane p into its ring slot
        {
            R* dstp = ringb + slot * PLANE;
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                const int r = ty + k * TY;
                if (r < LY) {
                    dstp[r * LX + lane] = pfa[k];
                    if (lane < 2 * H) dstp[r * LX + TX + lane] = pfb[k];
                }
            }
        }
        if constexpr (S::split) {
            // records of plane p - H + 1, the cz + 1 of the plane collided below
            const int qr = p - H + 1;
            if (qr >= za - 1 && qr <= zb) st.stage_store((qr - (za - 1)) % 3, ty, lane, pre);
        }
        __syncthreads();
        fetch(p + 1);
        st.stage_load(g, p - H + 2, x0, y0, ty, lane, pre);
        const int cz = p - H;
        if (cz < za) {
            // deviations of plane cz + 1 (the first collided plane's in the
            // last such iteration)
            st.template dev_load<W>(g, yc, max(cz + 1, 0), ln, pre);
            continue;  // uniform over the workgroup
        }
        const int s0 = (cz - (za - H)) % NP;
        const int sm = (s0 + NP - 1) % NP, sp = (s0 + 1) % NP;
        // N re-read each plane: the array offsets a N then stay scalar
        // arithmetic inside the loop instead of loop-invariant scalar
        // registers (which spill)
        unsigned Np = N;
        asm volatile("" : "+s"(Np));
        LeanPlane P;
        P.Np = Np;
        P.own_row = (unsigned)((cz * g.ny + yc) * g.nx);
        P.yc = yc;
        P.cz = cz;
        P.rs[0] = (cz - 1 - (za - 1)) % 3;
        P.rs[1] = (cz - (za - 1)) % 3;
        P.rs[2] = (cz + 1 - (za - 1)) % 3;
        // ---- pull (x, y, cz)
        R t[Q], d[Q];
        st.template pull<W, MV>(g, P, ln, pre, t, d);
        st.template dev_load<W>(g, yc, min(cz + 1, g.nz - 1), ln, pre);
        // ---- colour gradient from the ring: base at (ty + H - 1, lane + H - 1)
        R gx, gy, gz;
        {
            const int b = (ty + H - 1) * LX + lane + H - 1;
            const R* pm = ringb + sm * PLANE + b;
            const R* p0 = ringb + s0 * PLANE + b;
            const R* pp = ringb + sp * PLANE + b;
            R ax = R(0), ay = R(0), az = R(0);
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const R* pl = L::cz[i] < 0 ? pm : (L::cz[i] > 0 ? pp : p0);
                const R v = weight<R>(i) * pl[(1 + L::cy[i]) * LX + 1 + L::cx[i]];
                if (L::cx[i]) ax += L::cx[i] > 0 ? v : -v;
                if (L::cy[i]) ay += L::cy[i] > 0 ? v : -v;
                if (L::cz[i]) az += L::cz[i] > 0 ? v : -v;
            }
            gx = R(3) * ax;
            gy = R(3) * ay;
            gz = R(3) * az;
        }
        R Fx = c.fx, Fy = c.fy, Fz = c.fz;
        if (H > 1 && c.nc_range > 0) {
            PhiRing<R, TX, H> ring{ringb, LY};
            ring_near_contact<R, TX, H>(g, ring, s0, xc, yc, cz, ty + H, lane + H, gx, gy, gz, c, Fx, Fy, Fz);
        }
        SiteTotals<R> tot;
        collide<R, S::split>(t, d, gx, gy, gz, Fx, Fy, Fz, c, &tot);
        // ---- store (x, y, cz) and keep the values a later pull reads
        st.store(g, P, ln, t, d, tot, row_in && xin);
        if (ragged) {
            // lanes beyond the lattice hand nothing to their neighbours
            if (!xin) {
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    t[i] = -weight<R>(i);
                    d[i] = R(0);
                }
            }
        }
        // bounce-backs into this site: its own values, before the in-plane
        // group (off a moving wall, as the next pull reads them: plus the wall
        // term, shared by the site's own post-collision phase)
        {
            const bool ylo = W && g.wy && yc == 0, yhi = W && g.wy && yc == g.ny - 1;
            const bool zlo = W && g.wz && cz == 0, zhi = W && g.wz && cz == g.nz - 1;
            R ph = R(0);
            bool mv = false;
            if constexpr (W && MV) {
                mv = moving_next && (ylo || yhi || zlo || zhi || wall_xlo || wall_xhi);
                if (mv) {
                    if constexpr (S::split) {
                        ph = tot.phi;  // the phase the site's record holds
                    } else {
                        R st = R(0), sd = R(0);
                        for (int j = 0; j < Q; ++j) {
                            st += weight<R>(j) + t[j];
                            sd += d[j];
                        }
                        ph = sd / st;
                    }
                }
            }
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const bool ryz = (L::cy[i] > 0 && ylo) || (L::cy[i] < 0 && yhi) || (L::cz[i] > 0 && zlo) ||
                                 (L::cz[i] < 0 && zhi);
                if constexpr (W) {
                    const bool rx = (L::cx[i] > 0 && wall_xlo) || (L::cx[i] < 0 && wall_xhi);
                    if (ryz || rx) {
                        R tv = t[L::opp[i]], dv = d[L::opp[i]];
                        if (mv) {
                            const R add = wall_term<R>(g, i, xc, yc, cz);
                            tv += add;
                            dv += add * ph;
                        }
                        cur_rc += weight<R>(i) + tv;
                        cur_dn += dv;
                    }
                } else {
                    if (ryz) {
                        cur_rc += weight<R>(i) + t[L::opp[i]];
                        cur_dn += d[L::opp[i]];
                    }
                }
            }
        }
        // ---- hand the stored values of the directions with c_y != 0 to the
        // rows they stream to (LDS), w_i + t_i and d_i
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if (L::cy[i] == 0) continue;
            xrow[(2 * xch_slot(i)) * kLeanRowPad + 1 + lane] = weight<R>(i) + t[i];
            xrow[(2 * xch_slot(i) + 1) * kLeanRowPad + 1 + lane] = d[i];
        }
        if (edge_lo) xedge_own<R, TY, -1>(g, t, d, vs, ty, y, cz, za, zb, bd_lo, xf);
        if (edge_hi) xedge_own<R, TY, 1>(g, t, d, vs, ty, y, cz, za, zb, bd_hi, xf);
        __syncthreads();
        if (edge_lo) lean_xedge_rows<R, TY, -1>(g, xch, vs, ty, lane, nrows, y, cz, za, zb, bd_lo, xf);
        if (edge_hi) lean_xedge_rows<R, TY, 1>(g, xch, vs, ty, lane, nrows, y, cz, za, zb, bd_hi, xf);
        // value of direction i from the source (x - cx, y - cy) in plane cz:
        // 0 when the source is outside the tile or beyond a wall
        auto from = [&](int i, R& va, R& vd) {
            if (L::cy[i] != 0) {
                // (a source row beyond a y wall is also outside the tile's rows)
                const int ys = ty - L::cy[i];
                if (ys < 0 || ys >= nrows) {
                    va = R(0);
                    vd = R(0);
                    return;
                }
                const R* src = xch + ys * XROW + lane + 1 - L::cx[i];
                va = src[(2 * xch_slot(i)) * kLeanRowPad];
                vd = src[(2 * xch_slot(i) + 1) * kLeanRowPad];
            } else {
                const R a = weight<R>(i) + t[i];
                if (L::cx[i] > 0) {
                    va = from_left(a);
                    vd = from_left(d[i]);
                } else if (L::cx[i] < 0) {
                    va = from_right(a);
                    vd = from_right(d[i]);
                } else {
                    va = a;
                    vd = d[i];
                }
            }
        };
        // a site on an x or y face of the box keeps its own sums for the assembly
        const bool face_xy =
            lane == 0 || lane == TX - 1 || x == g.nx - 1 || ty == 0 || ty == TY - 1 || y == g.ny - 1;
        const bool site_in = row_in && xin;
        // destination cz - 1: sources in plane cz are its last group
        if (cz - 1 >= za) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if (L::cz[i] != -1) continue;
                R va, vd;
                from(i, va, vd);
                prev_rc += va;
                prev_dn += vd;
            }
            if (site_in) {
                const unsigned row = (unsigned)(((cz - 1) * g.ny + y) * g.nx);
                if (cz - 1 == za || face_xy)
                    res_store(Part2<R>{prev_dn, prev_rc}, array_res(part_out, N), (unsigned)x * sizeof(Part2<R>),
                              row * (unsigned)sizeof(Part2<R>));
                else
                    res_store_cached(prev_dn / prev_rc, array_res(phi_out, N), (unsigned)x * sizeof(R),
                                     row * (unsigned)sizeof(R));
            }
        }
        // destination cz: in-plane sources
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if (L::cz[i] != 0) continue;
            R va, vd;
            from(i, va, vd);
            cur_rc += va;
            cur_dn += vd;
        }
        // destination cz + 1: sources in plane cz are its first group
        R next_dn = R(0), next_rc = R(0);
        if (cz + 1 < zb) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if (L::cz[i] != 1) continue;
                R va, vd;
                from(i, va, vd);
                next_rc += va;
                next_dn += vd;
            }
        }
        prev_dn = cur_dn;
        prev_rc = cur_rc;
        cur_dn = next_dn;
        cur_rc = next_rc;
        // the chunk's last plane has no own sources above it
        if (cz == zb - 1 && site_in)
            res_store(Part2<R>{prev_dn, prev_rc}, array_res(part_out, N), (unsigned)x * sizeof(Part2<R>),
                      (unsigned)((cz * g.ny + y) * g.nx) * (unsigned)sizeof(Part2<R>));
        // no barrier here: the next staging overwrites ring slots that only
        // this plane's collide read, and every thread passed the barrier after
        // that collide before it gathers; the exchange rows are next written
        // after the next staging's barrier
    }
}

// LDS of a lean tile: phase-field ring, record ring (16-bit storage),
// exchange rows, x-face running sums.
template <typename S, int TY, int H>
__host__ __device__ constexpr size_t lean_lds_bytes() {
    using R = typename S::R;
    return ((phi_ring_bytes<R, kTX, H>(TY) + 15) & ~size_t(15)) + S::ring_bytes(TY) + lean_xch_bytes<R, TY>() +
           (size_t)2 * 3 * TY * sizeof(Part2<R>);
}

template <typename S, int TY, int H, bool W, bool MV>
__global__ __launch_bounds__(kTX * TY) void lean_kernel(Geom g, S st, Coeffs<typename S::R> c, FusedShape fs,
                                                       const Part2<typename S::R>* __restrict__ part_in,
                                                       Part2<typename S::R>* __restrict__ part_out,
                                                       int moving_next) {
    using R = typename S::R;
    extern __shared__ unsigned char lds_raw[];
    R* ringb = reinterpret_cast<R*>(lds_raw);
    size_t off = (phi_ring_bytes<R, kTX, H>(TY) + 15) & ~size_t(15);
    if constexpr (S::split) {
        st.ring = reinterpret_cast<f4*>(lds_raw + off);
        st.TY = TY;
    }
    off += S::ring_bytes(TY);
    R* xch = reinterpret_cast<R*>(lds_raw + off);
    Part2<R>* vs = reinterpret_cast<Part2<R>*>(lds_raw + off + lean_xch_bytes<R, TY>());
    int x0, y0, za, zb;
    tile_of_block(fs, kTX, g.nz, x0, y0, za, zb);
    lean_tile<S, TY, H, W, MV>(g, st, c, ringb, xch, vs, x0, y0, za, zb,
                           phi_of<kTX>(const_cast<Part2<R>*>(part_in), g), part_out, phi_of<kTX>(part_out, g),
                           moving_next);
}

}  // namespace lbm
