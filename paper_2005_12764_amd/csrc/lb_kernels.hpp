// lb_kernels.hpp -- population storage policies and the two-pass kernels
// (phase-field pass, then collide-and-stream pass), plus init, export,
// moments and compensated reductions.  Included by the translation units
// that instantiate and launch them.
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "d3q19.hpp"

namespace lbm {

// Lattice geometry.  Site index s = x + nx*(y + ny*z) (< 2^31).
struct Geom {
    int nx, ny, nz;
    int wx, wy, wz;  // 1 = halfway bounce-back walls on that axis
    int nxy;
    int N;
    int moving;      // some wall face moves (its reflections get a momentum term)
    double uw[6][3]; // wall face velocities, faces -x, +x, -y, +y, -z, +z
};

__device__ __forceinline__ void site_xyz(const Geom& g, int s, int& x, int& y, int& z) {
    z = s / g.nxy;
    const int r = s - z * g.nxy;
    y = r / g.nx;
    x = r - y * g.nx;
}

__device__ __forceinline__ int site_of(const Geom& g, int x, int y, int z) {
    return x + g.nx * (y + g.ny * z);
}

// Coordinate of the site a population arriving at v - c came from, for a
// unit step c: wraps on a periodic axis, flags a wall crossing.
__device__ __forceinline__ int step_back(int v, int c, int n, int wall, bool& bb) {
    int t = v - c;
    if (t < 0) {
        if (wall) bb = true;
        t += n;
    } else if (t >= n) {
        if (wall) bb = true;
        t -= n;
    }
    return t;
}

// Neighbour coordinate for the gradient stencil: wrap on periodic axes; on a
// wall axis the mirror image across the halfway wall.
__device__ __forceinline__ int stencil_coord(int v, int n, int wall) {
    if (v < 0) return wall ? -1 - v : v + n;
    if (v >= n) return wall ? 2 * n - 1 - v : v - n;
    return v;
}

// Pull source of direction i at (x,y,z): the upstream site, or the site
// itself in the opposite direction when the upstream site lies beyond a wall.
__device__ __forceinline__ int pull_source(const Geom& g, int i, int x, int y, int z, int s, int& d) {
    using L = Lattice;
    bool bb = false;
    const int xs = L::cx[i] ? step_back(x, L::cx[i], g.nx, g.wx, bb) : x;
    const int ys = L::cy[i] ? step_back(y, L::cy[i], g.ny, g.wy, bb) : y;
    const int zs = L::cz[i] ? step_back(z, L::cz[i], g.nz, g.wz, bb) : z;
    d = bb ? L::opp[i] : i;
    return bb ? s : site_of(g, xs, ys, zs);
}

// Per-site data of the pull: the site index, the index corrections of a
// periodic wrap on each side, and which sides are walls next to the site.
// Each direction's source is then a few selects and adds (the same result as
// pull_source, without its per-direction coordinate arithmetic).  Used by the
// 16-bit pulls, whose decode is arithmetic-bound; the raw pulls measured
// faster with pull_source.
struct Nbr {
    int s;
    int xm, xp, ym, yp, zm, zp;          // index change when the step wraps
    bool wxlo, wxhi, wylo, wyhi, wzlo, wzhi;  // a wall lies beyond this side
};
__device__ __forceinline__ Nbr nbr_of(const Geom& g, int s, int x, int y, int z) {
    Nbr n;
    n.s = s;
    n.xm = x == 0 ? g.nx : 0;
    n.xp = x == g.nx - 1 ? -g.nx : 0;
    n.ym = y == 0 ? g.nxy : 0;
    n.yp = y == g.ny - 1 ? -g.nxy : 0;
    n.zm = z == 0 ? g.N : 0;
    n.zp = z == g.nz - 1 ? -g.N : 0;
    n.wxlo = g.wx && x == 0;
    n.wxhi = g.wx && x == g.nx - 1;
    n.wylo = g.wy && y == 0;
    n.wyhi = g.wy && y == g.ny - 1;
    n.wzlo = g.wz && z == 0;
    n.wzhi = g.wz && z == g.nz - 1;
    return n;
}
__device__ __forceinline__ int nbr_source(const Geom& g, const Nbr& n, int i, int& d) {
    using L = Lattice;
    const bool bb = (L::cx[i] > 0 && n.wxlo) || (L::cx[i] < 0 && n.wxhi) || (L::cy[i] > 0 && n.wylo) ||
                    (L::cy[i] < 0 && n.wyhi) || (L::cz[i] > 0 && n.wzlo) || (L::cz[i] < 0 && n.wzhi);
    int src = n.s - (L::cx[i] + g.nx * L::cy[i] + g.nxy * L::cz[i]);
    if (L::cx[i] > 0) src += n.xm;
    if (L::cx[i] < 0) src += n.xp;
    if (L::cy[i] > 0) src += n.ym;
    if (L::cy[i] < 0) src += n.yp;
    if (L::cz[i] > 0) src += n.zm;
    if (L::cz[i] < 0) src += n.zp;
    d = bb ? L::opp[i] : i;
    return bb ? n.s : src;
}

// Moving-wall term of direction i arriving at (x,y,z) by reflection, in the
// compute type: 2 w_i (c_i . U)/c_s^2 summed over the wall faces the upstream
// site x - c_i lies beyond (reference density 1).
template <typename R>
__device__ __forceinline__ R wall_term(const Geom& g, int i, int x, int y, int z) {
    using L = Lattice;
    R cu = R(0);
    const int v[3] = {x - L::cx[i], y - L::cy[i], z - L::cz[i]};
    const int n[3] = {g.nx, g.ny, g.nz};
    const int w[3] = {g.wx, g.wy, g.wz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!w[a] || (v[a] >= 0 && v[a] < n[a])) continue;
        const double* U = g.uw[2 * a + (v[a] < 0 ? 0 : 1)];
        cu += R(L::cx[i]) * R(U[0]) + R(L::cy[i]) * R(U[1]) + R(L::cz[i]) * R(U[2]);
    }
    return R(6) * weight<R>(i) * cu;
}

// ---------------------------------------------------------------------------
// Storage policies.  pull() gathers the post-streaming populations of a site
// from the post-collision buffer of the previous step; store() writes the
// site's post-collision populations in place (aligned, coalesced).
// ---------------------------------------------------------------------------

// Raw storage of type T in shifted variables, t_i = f^r_i + f^b_i - w_i and
// d_i = f^r_i - f^b_i, as 19 arrays of (t_i, d_i) pairs: a direction's values
// of one site are 2 sizeof(T) contiguous bytes, so a pull or a store of a
// site moves 19 streams of pairs rather than 38 streams of single values.
// Consecutive arrays start raw_stride(N) pairs apart: the kRawPad unused pairs
// after each array keep the 19 streams of a site off a common power-of-two
// stride (which maps them onto the same HBM channels).
constexpr int kRawPad = 32;
__host__ __device__ constexpr size_t raw_stride(size_t N) { return N + kRawPad; }
template <typename T>
struct RawPair {
    typedef T type __attribute__((ext_vector_type(2)));
};
template <typename T>
__device__ __forceinline__ typename RawPair<T>::type raw_pair(const T* f, size_t N, int i, int s) {
    return *reinterpret_cast<const typename RawPair<T>::type*>(f + 2 * ((size_t)i * raw_stride(N) + s));
}
template <typename T>
__device__ __forceinline__ void raw_put(T* f, size_t N, int i, int s, T t, T d) {
    typename RawPair<T>::type v;
    v.x = t;
    v.y = d;
    *reinterpret_cast<typename RawPair<T>::type*>(f + 2 * ((size_t)i * raw_stride(N) + s)) = v;
}

// Raw storage policy.  MW: the lattice has moving walls (a separate
// instantiation, so resting-wall kernels carry none of that code).
template <typename T, bool MW = false>
struct RawPop {
    T* f;
    size_t N;

    template <typename R>
    __device__ __forceinline__ void pull(const Geom& g, int s, int x, int y, int z, R (&t)[Q],
                                         R (&d)[Q]) const {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int dir;
            const int src = pull_source(g, i, x, y, z, s, dir);
            const auto v = raw_pair(f, N, dir, src);
            t[i] = R(v.x);
            d[i] = R(v.y);
        }
        if constexpr (MW) {
            if (g.moving) add_wall_terms<R>(g, s, x, y, z, t, d);
        }
    }

    // Direction i of a pull whose source() gave (src, dir); no wall terms.
    template <typename R>
    __device__ __forceinline__ void pull_one(int i, int src, int dir, R& t, R& d) const {
        (void)i;
        const auto v = raw_pair(f, N, dir, src);
        t = R(v.x);
        d = R(v.y);
    }

    // The site's own post-collision x_r - x_b = sum d_j / sum (w_j + t_j) from
    // its stored values, summed in ascending direction.
    template <typename R>
    __device__ __forceinline__ R own_phase(int s) const {
        R st = R(0), sd = R(0);
        for (int j = 0; j < Q; ++j) {
            const auto v = raw_pair(f, N, j, s);
            st += weight<R>(j) + R(v.x);
            sd += R(v.y);
        }
        return sd / st;
    }
    // Moving-wall terms of the reflected directions, shared between the
    // components by the site's own post-collision rho_k/rho.
    template <typename R>
    __device__ void add_wall_terms(const Geom& g, int s, int x, int y, int z, R (&t)[Q], R (&d)[Q]) const {
        R ph = R(0);
        bool have = false;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            int dir;
            (void)pull_source(g, i, x, y, z, s, dir);
            if (dir == i) continue;
            if (!have) {
                ph = own_phase<R>(s);
                have = true;
            }
            const R add = wall_term<R>(g, i, x, y, z);
            t[i] += add;
            d[i] += add * ph;   // add x_r - add x_b
        }
    }
    template <typename R>
    __device__ __forceinline__ void store(int s, const R (&t)[Q], const R (&d)[Q],
                                          const SiteTotals<R>&) const {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            typename RawPair<T>::type v;
            v.x = T(t[i]);
            v.y = T(d[i]);
            __builtin_nontemporal_store(v, reinterpret_cast<typename RawPair<T>::type*>(f + 2 * ((size_t)i * raw_stride(N) + s)));
        }
    }
    // Store, and replace t, d by the values a later pull reads.
    template <typename R>
    __device__ __forceinline__ void store_as_read(int s, R (&t)[Q], R (&d)[Q], const SiteTotals<R>& tot) const {
        store(s, t, d, tot);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            t[i] = R(T(t[i]));
            d[i] = R(T(d[i]));
        }
    }
    static constexpr bool needs_totals = false;
    static constexpr bool ring = false;
    static constexpr bool moving = MW;
};

template <typename H>
struct Half;
template <>
struct Half<__half> {
    static __device__ __forceinline__ float to_f(__half h) { return __half2float(h); }
    static __device__ __forceinline__ __half from_f(float v) { return __float2half_rn(v); }
};
template <>
struct Half<__hip_bfloat16> {
    static __device__ __forceinline__ float to_f(__hip_bfloat16 h) { return __bfloat162float(h); }
    static __device__ __forceinline__ __hip_bfloat16 from_f(float v) { return __float2bfloat16(v); }
};

typedef float f4 __attribute__((ext_vector_type(4)));

// c_d . a for d = i (sg = 1) or its opposite (sg = -1), summed x, y, z from
// the non-zero components only, so that a value and its reflected reading
// round identically.
__device__ __forceinline__ float cdot(int i, float sg, float ax, float ay, float az) {
    using L = Lattice;
    float v = 0.0f;
    bool any = false;
    if (L::cx[i]) { v = L::cx[i] > 0 ? ax : -ax; any = true; }
    if (L::cy[i]) { const float b = L::cy[i] > 0 ? ay : -ay; v = any ? v + b : b; any = true; }
    if (L::cz[i]) { const float b = L::cz[i] > 0 ? az : -az; v = any ? v + b : b; }
    return sg * v;
}

// 16-bit moment-split storage.  Per site, 8 FP32 values rec[N][8] (two
// 16-byte vectors per site) of the post-collision state: density - 1, the
// momentum term J = 3 (j + F) of the equilibrium (3), the phase
// phi = x_r - x_b and the recolouring vector (3); per direction an array dev_i:
// the total post-collision population's deviation t_i from the reference
// w_i (drho + c_i . J) -- the equilibrium to first order in the velocity --
// times `scale`, in 16 bits (the second-order part of the equilibrium, of
// order u^2, is carried by the deviation with the non-equilibrium part).  The
// colour difference of direction i is phi (w_i + t_i) + 2 w_i (c_i . v)/|c_i|,
// exactly the form recolouring produces, so colour is carried in FP32.  The
// deviation arrays start dev_stride(N) values apart (kDevPad unused values
// after each, for the reason of raw_stride).  MW as for RawPop.
constexpr int kDevPad = 128;
__host__ __device__ constexpr size_t dev_stride(size_t N) { return N + kDevPad; }
template <typename H, bool MW = false>
struct SplitPop {
    float* rec;
    H* dev;
    size_t N;
    float scale, inv_scale;

    // Reference excess of direction i (read as d = i, sg = 1, or as its
    // opposite after a bounce-back, sg = -1) from the source record ra:
    // X = drho + c_i . J, so that f*_i - w_i = w_i X + deviation.  The
    // arithmetic is written out term by term so that every reading of a
    // stored value, and the store's own reading, rounds the same way.
    static __device__ __forceinline__ float excess(int i, float sg, const f4& ra) {
        return ra.x + cdot(i, sg, ra.y, ra.z, ra.w);
    }
    // Shifted variables t_i = f*_i - w_i and d_i = f^r_i - f^b_i from the
    // excess X, the 16-bit deviation and the colour part of the record rb.
    __device__ __forceinline__ void finish(int i, float sg, float X, const f4& rb, H dv16, float& tt,
                                           float& dd) const {
        const float w = weight<float>(i);
        tt = __builtin_fmaf(Half<H>::to_f(dv16), inv_scale, w * X);
        const float cv = cdot(i, sg, rb.y, rb.z, rb.w);
        dd = __builtin_fmaf(rb.x, w + tt, (2.0f * w * inv_clen<float>(i)) * cv);
    }
    template <typename R>
    __device__ __forceinline__ void decode(int i, int d, const f4& ra, const f4& rb, H dv16, R& t_i,
                                           R& d_i) const {
        const float sg = (d == i) ? 1.0f : -1.0f;
        float tt, dd;
        finish(i, sg, excess(i, sg, ra), rb, dv16, tt, dd);
        t_i = R(tt);
        d_i = R(dd);
    }

    template <typename R>
    __device__ __forceinline__ void pull(const Geom& g, int s, int x, int y, int z, R (&t)[Q],
                                         R (&d_)[Q]) const {
        const Nbr nb = nbr_of(g, s, x, y, z);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int d;
            const int src = nbr_source(g, nb, i, d);
            const f4 ra = *reinterpret_cast<const f4*>(rec + 8 * (size_t)src);
            const f4 rb = *reinterpret_cast<const f4*>(rec + 8 * (size_t)src + 4);
            decode<R>(i, d, ra, rb, dev[(size_t)d * dev_stride(N) + src], t[i], d_[i]);
        }
        if constexpr (MW) {
            if (g.moving) add_wall_terms<R>(g, s, x, y, z, rec[8 * (size_t)s + 4], t, d_);
        }
    }

    // Direction i of a pull whose source() gave (src, dir); no wall terms.
    template <typename R>
    __device__ __forceinline__ void pull_one(int i, int src, int dir, R& t, R& d) const {
        const f4 ra = *reinterpret_cast<const f4*>(rec + 8 * (size_t)src);
        const f4 rb = *reinterpret_cast<const f4*>(rec + 8 * (size_t)src + 4);
        decode<R>(i, dir, ra, rb, dev[(size_t)dir * dev_stride(N) + src], t, d);
    }

    // The site's own post-collision x_r - x_b: the phase of its record.
    template <typename R>
    __device__ __forceinline__ R own_phase(int s) const {
        return R(rec[8 * (size_t)s + 4]);
    }
    // Moving-wall terms of the reflected directions, shared by the site's own
    // post-collision phase phi (from its record): add x_r - add x_b.
    template <typename R>
    __device__ void add_wall_terms(const Geom& g, int s, int x, int y, int z, float phi, R (&t)[Q],
                                   R (&d)[Q]) const {
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            int dir;
            (void)pull_source(g, i, x, y, z, s, dir);
            if (dir == i) continue;
            const R add = wall_term<R>(g, i, x, y, z);
            t[i] += add;
            d[i] += add * R(phi);
        }
    }

    // As pull(), with the source records taken from an LDS ring that holds
    // the records of planes z-1, z, z+1 around the tile (one-site halo):
    // `ring[k]` points at the plane of z - 1 + k, (ly, lx) is the site's
    // position in the ring plane, LXR its row length.
    template <typename R>
    __device__ __forceinline__ void pull_ring(const Geom& g, int s, int x, int y, int z, R (&t)[Q],
                                              R (&d_)[Q], const f4* const (&ring)[3], int ly, int lx,
                                              int LXR, int half) const {
        using L = Lattice;
        const Nbr nb = nbr_of(g, s, x, y, z);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int d;
            const int src = nbr_source(g, nb, i, d);
            const bool bb = (d != i);
            const f4* pl = bb ? ring[1] : ring[1 - L::cz[i]];
            const int pos = bb ? (ly * LXR + lx) : ((ly - L::cy[i]) * LXR + lx - L::cx[i]);
            decode<R>(i, d, pl[pos], pl[half + pos], dev[(size_t)d * dev_stride(N) + src], t[i], d_[i]);
        }
        if constexpr (MW) {
            const float phi_own = ring[1][half + ly * LXR + lx].x;
            if (g.moving) add_wall_terms<R>(g, s, x, y, z, phi_own, t, d_);
        }
    }

    template <typename R>
    __device__ __forceinline__ void store(int s, const R (&t)[Q], const R (&d)[Q],
                                          const SiteTotals<R>& tot) const {
        R tc[Q], dc[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            tc[i] = t[i];
            dc[i] = d[i];
        }
        store_as_read(s, tc, dc, tot);
    }
    // Store, and replace t, d by the values a later pull decodes (exactly).
    template <typename R>
    __device__ __forceinline__ void store_as_read(int s, R (&t)[Q], R (&d)[Q], const SiteTotals<R>& tot) const {
        const f4 ra = {float(tot.drho), float(tot.jx), float(tot.jy), float(tot.jz)};
        const f4 rb = {float(tot.phi), float(tot.vx), float(tot.vy), float(tot.vz)};
        __builtin_nontemporal_store(ra, reinterpret_cast<f4*>(rec + 8 * (size_t)s));
        __builtin_nontemporal_store(rb, reinterpret_cast<f4*>(rec + 8 * (size_t)s + 4));
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const float X = excess(i, 1.0f, ra);
            // deviation of f*_i - w_i = t_i from w_i X
            const H h = Half<H>::from_f((float(t[i]) - weight<float>(i) * X) * scale);
            dev[(size_t)i * dev_stride(N) + s] = h;
            float tt, dd;
            finish(i, 1.0f, X, rb, h, tt, dd);
            t[i] = R(tt);
            d[i] = R(dd);
        }
    }
    static constexpr bool needs_totals = true;
    static constexpr bool ring = true;
    static constexpr bool moving = MW;
};

// Minimum waves per SIMD the step kernels ask the compiler for, per storage.
// The 16-bit decode keeps the 19 source records in flight (~190 VGPRs, two
// waves per SIMD); asking for more waves makes the compiler spill, which
// measured 3x slower, so no bound is imposed by default.
#ifndef LB_SPLIT_WAVES
#define LB_SPLIT_WAVES 1
#endif
template <typename S>
struct Occupancy {
    static constexpr int waves = 1;
};
template <typename H, bool MW>
struct Occupancy<SplitPop<H, MW>> {
    static constexpr int waves = LB_SPLIT_WAVES;
};
template <typename A, typename B>
constexpr int waves_of() {
    return Occupancy<A>::waves > Occupancy<B>::waves ? Occupancy<A>::waves : Occupancy<B>::waves;
}

// ---------------------------------------------------------------------------
// Phase field and colour gradient.
// ---------------------------------------------------------------------------

// G(x) = 3 sum_i w_i phi(x + c_i) c_i, mirror sites beyond walls.
template <typename R>
__device__ __forceinline__ void gradient(const Geom& g, const R* __restrict__ phi, int x, int y,
                                         int z, R& gx, R& gy, R& gz) {
    using L = Lattice;
    R ax = R(0), ay = R(0), az = R(0);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int xn = L::cx[i] ? stencil_coord(x + L::cx[i], g.nx, g.wx) : x;
        const int yn = L::cy[i] ? stencil_coord(y + L::cy[i], g.ny, g.wy) : y;
        const int zn = L::cz[i] ? stencil_coord(z + L::cz[i], g.nz, g.wz) : z;
        const R p = weight<R>(i) * phi[site_of(g, xn, yn, zn)];
        if (L::cx[i]) ax += L::cx[i] > 0 ? p : -p;
        if (L::cy[i]) ay += L::cy[i] > 0 ? p : -p;
        if (L::cz[i]) az += L::cz[i] > 0 ? p : -p;
    }
    gx = R(3) * ax;
    gy = R(3) * ay;
    gz = R(3) * az;
}

__device__ __forceinline__ int wrap_any(int v, int n) {
    int r = v % n;
    return r < 0 ? r + n : r;
}

// Near-contact force A_h(h) G at (x,y,z): interface sites probe their outward
// normal ray x + round(k n), k = 1..K, for an interface site whose gradient
// opposes G; a sample beyond a wall ends the probe.
template <typename R>
__device__ __forceinline__ void near_contact(const Geom& g, const R* __restrict__ phi, int x, int y,
                                             int z, R gx, R gy, R gz, const Coeffs<R>& c, R& Fx,
                                             R& Fy, R& Fz) {
    const R g2 = gx * gx + gy * gy + gz * gz;
    if (!at_least(g2, c.g_iface, c.g_iface2)) return;
    const R inv_gm = inv_norm(g2);
    const R nx = -gx * inv_gm, ny = -gy * inv_gm, nz = -gz * inv_gm;
    int h = 0;
    for (int k = 1; k <= c.nc_range; ++k) {
        int px = x + (int)round(R(k) * nx);
        int py = y + (int)round(R(k) * ny);
        int pz = z + (int)round(R(k) * nz);
        if (g.wx) { if (px < 0 || px >= g.nx) break; } else px = wrap_any(px, g.nx);
        if (g.wy) { if (py < 0 || py >= g.ny) break; } else py = wrap_any(py, g.ny);
        if (g.wz) { if (pz < 0 || pz >= g.nz) break; } else pz = wrap_any(pz, g.nz);
        R qx, qy, qz;
        gradient<R>(g, phi, px, py, pz, qx, qy, qz);
        const R q2 = qx * qx + qy * qy + qz * qz;
        const R dot = qx * gx + qy * gy + qz * gz;
        if (dot < R(0) && at_least(q2, c.g_iface, c.g_iface2)) {
            h = k;
            break;
        }
    }
    const R ah = nc_amplitude<R>(h, c);
    Fx += ah * gx;
    Fy += ah * gy;
    Fz += ah * gz;
}

// ---------------------------------------------------------------------------
// Two-pass step.
// ---------------------------------------------------------------------------

// phi = (rho_r - rho_b)/rho = sum_i d_i / sum_i (w_i + t_i), the density
// summed as the collision sums it for the colour split (exactly +-1 in a
// pure component).
template <typename R>
__device__ __forceinline__ R phase_of(const R (&t)[Q], const R (&d)[Q]) {
    R rc = R(0), sd = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        rc += weight<R>(i) + t[i];
        sd += d[i];
    }
    return sd / rc;
}

// Pass 1: phi = (rho_r - rho_b)/rho of the post-streaming state.
template <typename R, typename Src>
__global__ __launch_bounds__(256, Occupancy<Src>::waves) void phase_kernel(Geom g, Src src, R* __restrict__ phi) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.N) return;
    int x, y, z;
    site_xyz(g, s, x, y, z);
    R t[Q], d[Q];
    src.pull(g, s, x, y, z, t, d);
    phi[s] = phase_of(t, d);
}

// Pass 2: pull, colour gradient, near-contact, collision, store.
template <typename R, typename Src, typename Dst>
__global__ __launch_bounds__(256, (waves_of<Src, Dst>())) void collide_kernel(Geom g, Src src, Dst dst,
                                                      const R* __restrict__ phi, Coeffs<R> c) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.N) return;
    int x, y, z;
    site_xyz(g, s, x, y, z);
    R t[Q], d[Q];
    src.pull(g, s, x, y, z, t, d);
    R gx, gy, gz;
    gradient<R>(g, phi, x, y, z, gx, gy, gz);
    R Fx = c.fx, Fy = c.fy, Fz = c.fz;
    if (c.nc_range > 0 && c.nc_strength != R(0)) near_contact<R>(g, phi, x, y, z, gx, gy, gz, c, Fx, Fy, Fz);
    SiteTotals<R> tot;
    collide<R>(t, d, gx, gy, gz, Fx, Fy, Fz, c, &tot);
    dst.store(s, t, d, tot);
}

// ---------------------------------------------------------------------------
// Init / import (into raw storage), export, moments.
// ---------------------------------------------------------------------------

// Post-collision buffer whose pull gives f^eq(rho_k, u) at every site:
// buf_j(y) = f^eq_j(y + c_j), or f^eq_opp(j)(y) when y + c_j lies beyond a wall.
template <typename T, typename In>
__global__ __launch_bounds__(256) void init_raw_kernel(Geom g, T* __restrict__ f, const In* rr,
                                                       const In* rb, const In* u) {
    using L = Lattice;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.N) return;
    int x, y, z;
    site_xyz(g, s, x, y, z);
    const size_t N = (size_t)g.N;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        // the target of direction j from s is where the population streams to
        bool bb = false;
        const int xt = L::cx[j] ? step_back(x, -L::cx[j], g.nx, g.wx, bb) : x;
        const int yt = L::cy[j] ? step_back(y, -L::cy[j], g.ny, g.wy, bb) : y;
        const int zt = L::cz[j] ? step_back(z, -L::cz[j], g.nz, g.wz, bb) : z;
        const int t = bb ? s : site_of(g, xt, yt, zt);
        const int d = bb ? L::opp[j] : j;
        double ux = 0, uy = 0, uz = 0;
        if (u) {
            ux = double(u[t]);
            uy = double(u[N + t]);
            uz = double(u[2 * N + t]);
        }
        // f^eq_d(rho_k, u) = rho_k w (1 + q): t = w (rho - 1 + rho q), d = (rho_r - rho_b) w (1 + q)
        const double cu = L::cx[d] * ux + L::cy[d] * uy + L::cz[d] * uz;
        const double uu = ux * ux + uy * uy + uz * uz;
        const double q = 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
        const double w = weight<double>(d);
        const double a = double(rr[t]), b = double(rb[t]);
        raw_put(f, N, j, s, T(w * ((a + b - 1.0) + (a + b) * q)), T((a - b) * w * (1.0 + q)));
    }
}

// Import of post-streaming populations fin[2][19][N] into raw post-collision
// storage (the inverse of the pull).
template <typename T, typename In>
__global__ __launch_bounds__(256) void import_raw_kernel(Geom g, T* __restrict__ f,
                                                         const In* __restrict__ fin) {
    using L = Lattice;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.N) return;
    int x, y, z;
    site_xyz(g, s, x, y, z);
    const size_t N = (size_t)g.N;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        bool bb = false;
        const int xt = L::cx[j] ? step_back(x, -L::cx[j], g.nx, g.wx, bb) : x;
        const int yt = L::cy[j] ? step_back(y, -L::cy[j], g.ny, g.wy, bb) : y;
        const int zt = L::cz[j] ? step_back(z, -L::cz[j], g.nz, g.wz, bb) : z;
        const int t = bb ? s : site_of(g, xt, yt, zt);
        const int d = bb ? L::opp[j] : j;
        const double a = double(fin[(size_t)d * N + t]), b = double(fin[(size_t)(Q + d) * N + t]);
        raw_put(f, N, j, s, T((a + b) - weight<double>(d)), T(a - b));
    }
}

// Export of the post-streaming populations.
template <typename R, typename Src, typename Out>
__global__ __launch_bounds__(256) void export_kernel(Geom g, Src src, Out* __restrict__ out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.N) return;
    int x, y, z;
    site_xyz(g, s, x, y, z);
    // decoded in FP64 whatever the storage, so that f^r + f^b - w and
    // f^r - f^b of the export reproduce the stored values
    double t[Q], d[Q];
    src.pull(g, s, x, y, z, t, d);
    const size_t N = (size_t)g.N;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        double fr, fb;
        from_shifted<double>(i, t[i], d[i], fr, fb);
        out[(size_t)i * N + s] = Out(fr);
        out[(size_t)(Q + i) * N + s] = Out(fb);
    }
}

// Moments rho_r, rho_b, j of the post-streaming state (any output may be null).
template <typename R, typename Src, typename Out>
__global__ __launch_bounds__(256) void moments_kernel(Geom g, Src src, Out* rr_out, Out* rb_out,
                                                      Out* j_out) {
    using L = Lattice;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.N) return;
    int x, y, z;
    site_xyz(g, s, x, y, z);
    R t[Q], d[Q];
    src.pull(g, s, x, y, z, t, d);
    R st = R(0), sd = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        st += t[i];
        sd += d[i];
        if (L::cx[i]) jx += L::cx[i] > 0 ? t[i] : -t[i];
        if (L::cy[i]) jy += L::cy[i] > 0 ? t[i] : -t[i];
        if (L::cz[i]) jz += L::cz[i] > 0 ? t[i] : -t[i];
    }
    const R rr = R(0.5) * (R(1) + st + sd), rb = R(0.5) * (R(1) + st - sd);
    const size_t N = (size_t)g.N;
    if (rr_out) rr_out[s] = Out(rr);
    if (rb_out) rb_out[s] = Out(rb);
    if (j_out) {
        j_out[s] = Out(jx);
        j_out[N + s] = Out(jy);
        j_out[2 * N + s] = Out(jz);
    }
}

// Initial densities from a droplet list: phi0 = max(background,
// max_j tanh((R_j - d_j)/width)) over droplets with d_j <= R_j + 6 width
// (periodic minimum image on periodic axes), rho_r = rho0 (1 + phi0)/2,
// rho_b = rho0 (1 - phi0)/2.
__device__ __forceinline__ double min_image(double d, int n, int wall) {
    return wall ? d : d - double(n) * rint(d / double(n));
}

static __global__ __launch_bounds__(256) void droplet_fields_kernel(Geom g, const double* __restrict__ cen,
                                                                   const double* __restrict__ rad, int n,
                                                                   double width, double background, double rho0,
                                                                   double* __restrict__ rr, double* __restrict__ rb) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.N) return;
    int x, y, z;
    site_xyz(g, s, x, y, z);
    double phi = background;
    for (int j = 0; j < n; ++j) {
        const double R = rad[j];
        const double dx = min_image(double(x) - cen[3 * j], g.nx, g.wx);
        const double dy = min_image(double(y) - cen[3 * j + 1], g.ny, g.wy);
        const double dz = min_image(double(z) - cen[3 * j + 2], g.nz, g.wz);
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r <= R + 6.0 * width) phi = fmax(phi, tanh((R - r) / width));
    }
    rr[s] = rho0 * (1.0 + phi) / 2.0;
    rb[s] = rho0 * (1.0 - phi) / 2.0;
}

// ---------------------------------------------------------------------------
// Deterministic compensated FP64 totals.
// ---------------------------------------------------------------------------
constexpr int NTOT = 7;  // red mass, blue mass, jx, jy, jz, kinetic energy, bad sites

struct Neu {
    double s, c;
};
__device__ __forceinline__ void neu_add(Neu& a, double x) {
    const double t = a.s + x;
    if (fabs(a.s) >= fabs(x))
        a.c += (a.s - t) + x;
    else
        a.c += (x - t) + a.s;
    a.s = t;
}
__device__ __forceinline__ void neu_merge(Neu& a, const Neu& b) {
    neu_add(a, b.s);
    a.c += b.c;
}

// Block-level fixed-order reduction: wave shuffles, then the 4 wave results
// through LDS in wave order.  Every thread must call it.
__device__ __forceinline__ void block_reduce(Neu (&acc)[NTOT], Neu* lds /* [4][NTOT] */) {
#pragma unroll
    for (int q = 0; q < NTOT; ++q) {
        for (int off = 32; off >= 1; off >>= 1) {
            Neu o;
            o.s = __shfl_down(acc[q].s, off, 64);
            o.c = __shfl_down(acc[q].c, off, 64);
            neu_merge(acc[q], o);
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int q = 0; q < NTOT; ++q) lds[wave * NTOT + q] = acc[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < NTOT; ++q) {
            Neu r = lds[q];
            for (int w = 1; w < (int)(blockDim.x >> 6); ++w) neu_merge(r, lds[w * NTOT + q]);
            acc[q] = r;
        }
    }
}

template <typename R, typename Src>
__global__ __launch_bounds__(256) void totals_kernel(Geom g, Src src, Neu* __restrict__ partial) {
    using L = Lattice;
    __shared__ Neu lds[4 * NTOT];
    Neu acc[NTOT];
#pragma unroll
    for (int q = 0; q < NTOT; ++q) acc[q] = Neu{0.0, 0.0};
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < g.N; s += gridDim.x * blockDim.x) {
        int x, y, z;
        site_xyz(g, s, x, y, z);
        R t[Q], d[Q];
        src.pull(g, s, x, y, z, t, d);
        double st = 0, sd = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            st += double(t[i]);
            sd += double(d[i]);
            const double ti = double(t[i]);
            if (L::cx[i]) jx += L::cx[i] > 0 ? ti : -ti;
            if (L::cy[i]) jy += L::cy[i] > 0 ? ti : -ti;
            if (L::cz[i]) jz += L::cz[i] > 0 ? ti : -ti;
        }
        const double rr = 0.5 * (1.0 + st + sd), rb = 0.5 * (1.0 + st - sd);
        const double rho = rr + rb;
        const bool bad = !(rho > 0.0) || !isfinite(rho) || !isfinite(jx) || !isfinite(jy) ||
                         !isfinite(jz);
        neu_add(acc[0], rr);
        neu_add(acc[1], rb);
        neu_add(acc[2], jx);
        neu_add(acc[3], jy);
        neu_add(acc[4], jz);
        neu_add(acc[5], bad ? 0.0 : 0.5 * (jx * jx + jy * jy + jz * jz) / rho);
        neu_add(acc[6], bad ? 1.0 : 0.0);
    }
    block_reduce(acc, lds);
    if (threadIdx.x == 0)
        for (int q = 0; q < NTOT; ++q) partial[blockIdx.x * NTOT + q] = acc[q];
}

// One block folds the per-block partials in block order.
static __global__ __launch_bounds__(256) void totals_final_kernel(const Neu* __restrict__ partial, int nblocks,
                                                           double* __restrict__ out) {
    __shared__ Neu lds[4 * NTOT];
    Neu acc[NTOT];
#pragma unroll
    for (int q = 0; q < NTOT; ++q) acc[q] = Neu{0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int q = 0; q < NTOT; ++q) neu_merge(acc[q], partial[b * NTOT + q]);
    block_reduce(acc, lds);
    if (threadIdx.x == 0)
        for (int q = 0; q < NTOT; ++q) {
            out[2 * q] = acc[q].s;
            out[2 * q + 1] = acc[q].c;
        }
}

}  // namespace lbm
