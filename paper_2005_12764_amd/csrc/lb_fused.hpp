// lb_fused.hpp -- z-marching tile kernels of the two-pass step.
//
// A workgroup owns a tile of TX x TY columns and marches it through a chunk of
// z-planes, keeping the phase field phi in an LDS ring of 2H+1 planes (tile
// plus a halo of H = K + 1 sites, K = near-contact range).  The plane H behind
// the newest one then has phi on every site its colour gradient and the
// gradients along its near-contact probes can reach, and is collided.  phi
// comes from the phase pass's array, so each site's populations are read once
// by the collide pass; for 16-bit moment-split storage the per-site FP32
// records of planes z-1..z+1 (tile plus one site) are staged in a second LDS
// ring so that the 19 source records of a pull come from LDS.  The phase pass
// of 16-bit storage marches the same tiles with the record ring only.
#pragma once
#include "lb_kernels.hpp"

namespace lbm {

struct FusedShape {
    int TY;        // tile rows (TX is a template constant)
    int TZ;        // planes per z chunk
    int tiles_x, tiles_y, chunks;
    int nblocks;   // tiles_x * tiles_y * chunks
};

// Coordinate of an LDS position along one axis: wrap on periodic axes, mirror
// (then clamp, for positions far beyond a tiny lattice) on wall axes.
__device__ __forceinline__ int halo_coord(int v, int n, int wall) {
    if (v >= 0 && v < n) return v;
    if (wall) {
        int m = v < 0 ? -1 - v : 2 * n - 1 - v;
        return m < 0 ? 0 : (m >= n ? n - 1 : m);
    }
    int r = v % n;
    return r < 0 ? r + n : r;
}

template <typename R, int TX, int H>
struct PhiRing {
    static constexpr int LX = TX + 2 * H;
    static constexpr int NP = 2 * H + 1;
    R* base;
    int LY;
    __device__ __forceinline__ R* plane(int slot) const { return base + (size_t)slot * LY * LX; }
};

// Ring of 3 planes of 16-bit-storage records (2 x f4 per site), tile plus one
// site around it; each plane holds the first f4 of every site, then the
// second (consecutive lanes read consecutive 16-byte words: no bank conflicts).
template <int TX>
struct RecRing {
    static constexpr int LX = TX + 2;
    f4* base;
    int LY;
    __device__ __forceinline__ f4* plane(int slot) const { return base + (size_t)slot * LY * LX * 2; }
    __device__ __forceinline__ int half() const { return LY * LX; }
};

template <typename R, int TX, int H>
__host__ __device__ constexpr size_t phi_ring_bytes(int TY) {
    return (size_t)(2 * H + 1) * (TY + 2 * H) * (TX + 2 * H) * sizeof(R);
}
template <int TX>
__host__ __device__ constexpr size_t rec_ring_bytes(int TY) {
    return (size_t)3 * (TY + 2) * (TX + 2) * 2 * sizeof(f4);
}

// Copy the records of plane q (tile plus one site) into a ring slot.
template <typename Src, int TX>
__device__ __forceinline__ void load_rec_plane(const Geom& g, const Src& src, const RecRing<TX>& rr, int slot,
                                               int x0, int y0, int q) {
    constexpr int LX = RecRing<TX>::LX;
    f4* dstp = rr.plane(slot);
    const int zz = halo_coord(q, g.nz, g.wz);
    for (int k = threadIdx.x; k < rr.LY * LX; k += blockDim.x) {
        const int ly = k / LX, lx = k - ly * LX;
        const int xx = halo_coord(x0 - 1 + lx, g.nx, g.wx);
        const int yy = halo_coord(y0 - 1 + ly, g.ny, g.wy);
        const size_t s = (size_t)site_of(g, xx, yy, zz);
        const f4 a = *reinterpret_cast<const f4*>(src.rec + 8 * s);
        const f4 b = *reinterpret_cast<const f4*>(src.rec + 8 * s + 4);
        dstp[k] = a;
        dstp[rr.half() + k] = b;
    }
}

// G at LDS position (ly, lx) of the plane in `slot`, from the three ring planes
// around it: 3 sum_i w_i phi(x + c_i) c_i.
template <typename R, int TX, int H>
__device__ __forceinline__ void lds_gradient(const PhiRing<R, TX, H>& ring, int sm, int s0, int sp,
                                             int ly, int lx, R& gx, R& gy, R& gz) {
    using L = Lattice;
    constexpr int LX = PhiRing<R, TX, H>::LX;
    const R* pm = ring.plane(sm);
    const R* p0 = ring.plane(s0);
    const R* pp = ring.plane(sp);
    R ax = R(0), ay = R(0), az = R(0);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const R* pl = L::cz[i] < 0 ? pm : (L::cz[i] > 0 ? pp : p0);
        const R v = weight<R>(i) * pl[(ly + L::cy[i]) * LX + lx + L::cx[i]];
        if (L::cx[i]) ax += L::cx[i] > 0 ? v : -v;
        if (L::cy[i]) ay += L::cy[i] > 0 ? v : -v;
        if (L::cz[i]) az += L::cz[i] > 0 ? v : -v;
    }
    gx = R(3) * ax;
    gy = R(3) * ay;
    gz = R(3) * az;
}

// Near-contact force from the phi ring (probe samples within K < H sites).
template <typename R, int TX, int H>
__device__ __forceinline__ void ring_near_contact(const Geom& g, const PhiRing<R, TX, H>& ring, int s0, int x,
                                                  int y, int z, int ly, int lx, R gx, R gy, R gz,
                                                  const Coeffs<R>& c, R& Fx, R& Fy, R& Fz) {
    constexpr int NP = 2 * H + 1;
    const R g2 = gx * gx + gy * gy + gz * gz;
    if (!at_least(g2, c.g_iface, c.g_iface2)) return;
    const R inv_gm = inv_norm(g2);
    const R nx = -gx * inv_gm, ny = -gy * inv_gm, nz = -gz * inv_gm;
    int h = 0;
    for (int k = 1; k <= c.nc_range && k < H; ++k) {
        const int ox = (int)round(R(k) * nx);
        const int oy = (int)round(R(k) * ny);
        const int oz = (int)round(R(k) * nz);
        // a probe sample beyond a wall ends the probe
        if (g.wx && (x + ox < 0 || x + ox >= g.nx)) break;
        if (g.wy && (y + oy < 0 || y + oy >= g.ny)) break;
        if (g.wz && (z + oz < 0 || z + oz >= g.nz)) break;
        const int t0 = (s0 + oz + NP) % NP;
        R qx, qy, qz;
        lds_gradient<R, TX, H>(ring, (t0 + NP - 1) % NP, t0, (t0 + 1) % NP, ly + oy, lx + ox, qx, qy, qz);
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

// One tile of the collide pass: columns [x0, x0+TX) x [y0, y0+TY), planes
// [za, zb), phi from the phase pass and, for storage with per-site records,
// the records of planes z-1..z+1 in `rr`.  Every thread of the workgroup must
// call it (it holds barriers).
template <typename R, typename Src, typename Dst, int TX, int H>
__device__ __forceinline__ void fused_tile(const Geom& g, const Src& src, const Dst& dst, const Coeffs<R>& c,
                                           const PhiRing<R, TX, H>& ring, int TY, int x0, int y0, int za,
                                           int zb, const R* __restrict__ phi_in, const RecRing<TX>& rr) {
    constexpr int LX = TX + 2 * H;
    constexpr int NP = 2 * H + 1;
    const int LY = ring.LY;
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    for (int p = za - H; p < zb + H; ++p) {
        const int slot = (p - (za - H)) % NP;
        // ---- phase field of plane p on the tile and its halo
        {
            R* dstp = ring.plane(slot);
            const int zz = halo_coord(p, g.nz, g.wz);
            for (int q = tid; q < LY * LX; q += nt) {
                const int ly = q / LX, lx = q - ly * LX;
                const int xx = halo_coord(x0 - H + lx, g.nx, g.wx);
                const int yy = halo_coord(y0 - H + ly, g.ny, g.wy);
                dstp[q] = phi_in[site_of(g, xx, yy, zz)];
            }
        }
        if constexpr (Src::ring) {
            // records of plane cz + 1 (planes cz - 1 and cz came in earlier)
            const int qr = p - H + 1;
            if (qr >= za - 1 && qr <= zb) load_rec_plane<Src, TX>(g, src, rr, (qr - za + 1) % 3, x0, y0, qr);
        }
        __syncthreads();
        // ---- collide plane cz = p - H: its phi neighbourhood is complete
        const int cz = p - H;
        if (cz >= za) {
            const int s0 = (cz - (za - H)) % NP;
            const int sm = (s0 + NP - 1) % NP, sp = (s0 + 1) % NP;
            for (int q = tid; q < TY * TX; q += nt) {
                const int ty = q / TX, tx = q - ty * TX;
                const int x = x0 + tx, y = y0 + ty;
                if (x >= g.nx || y >= g.ny) continue;
                const int s = site_of(g, x, y, cz);
                R t[Q], d[Q];
                if constexpr (Src::ring) {
                    const f4* const planes[3] = {rr.plane((cz - za) % 3), rr.plane((cz - za + 1) % 3),
                                                 rr.plane((cz - za + 2) % 3)};
                    src.pull_ring(g, s, x, y, cz, t, d, planes, ty + 1, tx + 1, RecRing<TX>::LX, rr.half());
                } else {
                    src.pull(g, s, x, y, cz, t, d);
                }
                const int ly = ty + H, lx = tx + H;
                R gx, gy, gz;
                lds_gradient<R, TX, H>(ring, sm, s0, sp, ly, lx, gx, gy, gz);
                R Fx = c.fx, Fy = c.fy, Fz = c.fz;
                if (H > 1 && c.nc_range > 0)
                    ring_near_contact<R, TX, H>(g, ring, s0, x, y, cz, ly, lx, gx, gy, gz, c, Fx, Fy, Fz);
                SiteTotals<R> tot;
                collide<R>(t, d, gx, gy, gz, Fx, Fy, Fz, c, &tot);
                dst.store(s, t, d, tot);
            }
        }
        __syncthreads();
    }
}

// Phase pass over one tile: phi of planes [za, zb).  Storage with per-site
// records stages planes z-1..z+1 in the record ring; raw storage pulls
// directly.
template <typename R, typename Src, int TX>
__device__ __forceinline__ void phase_tile(const Geom& g, const Src& src, R* __restrict__ phi, const RecRing<TX>& rr,
                                           int TY, int x0, int y0, int za, int zb) {
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    if constexpr (Src::ring) {
        for (int q = za - 1; q <= zb; ++q) {
            load_rec_plane<Src, TX>(g, src, rr, (q - za + 1) % 3, x0, y0, q);
            __syncthreads();
            const int cz = q - 1;
            if (cz >= za) {
                const f4* const planes[3] = {rr.plane((cz - za) % 3), rr.plane((cz - za + 1) % 3),
                                             rr.plane((cz - za + 2) % 3)};
                for (int k = tid; k < TY * TX; k += nt) {
                    const int ty = k / TX, tx = k - ty * TX;
                    const int x = x0 + tx, y = y0 + ty;
                    if (x >= g.nx || y >= g.ny) continue;
                    const int s = site_of(g, x, y, cz);
                    R t[Q], d[Q];
                    src.pull_ring(g, s, x, y, cz, t, d, planes, ty + 1, tx + 1, RecRing<TX>::LX, rr.half());
                    phi[s] = phase_of(t, d);
                }
            }
            __syncthreads();
        }
    } else {
        for (int cz = za; cz < zb; ++cz)
            for (int k = tid; k < TY * TX; k += nt) {
                const int ty = k / TX, tx = k - ty * TX;
                const int x = x0 + tx, y = y0 + ty;
                if (x >= g.nx || y >= g.ny) continue;
                const int s = site_of(g, x, y, cz);
                R t[Q], d[Q];
                src.pull(g, s, x, y, cz, t, d);
                phi[s] = phase_of(t, d);
            }
    }
}

// Tile of this workgroup: workgroups are dealt round-robin to the 8 XCDs, so
// each XCD gets a contiguous run of tiles (neighbouring tiles share halo rows
// in its L2).
__device__ __forceinline__ void tile_of_block(const FusedShape& fs, int TX, int nz, int& x0, int& y0, int& za,
                                              int& zb) {
    int b = blockIdx.x;
    if ((fs.nblocks & 7) == 0) b = (b & 7) * (fs.nblocks >> 3) + (b >> 3);
    const int tile = b % (fs.tiles_x * fs.tiles_y);
    const int chunk = b / (fs.tiles_x * fs.tiles_y);
    x0 = (tile % fs.tiles_x) * TX;
    y0 = (tile / fs.tiles_x) * fs.TY;
    za = chunk * fs.TZ;
    zb = min(za + fs.TZ, nz);
}

template <typename R, typename Src, typename Dst, int TX, int H>
__global__ __launch_bounds__(256, (waves_of<Src, Dst>())) void fused_kernel(Geom g, Src src, Dst dst, Coeffs<R> c,
                                                                            FusedShape fs, const R* __restrict__ phi_in) {
    extern __shared__ unsigned char lds_raw[];
    PhiRing<R, TX, H> ring{reinterpret_cast<R*>(lds_raw), fs.TY + 2 * H};
    RecRing<TX> rr{reinterpret_cast<f4*>(lds_raw + ((phi_ring_bytes<R, TX, H>(fs.TY) + 15) & ~size_t(15))), fs.TY + 2};
    int x0, y0, za, zb;
    tile_of_block(fs, TX, g.nz, x0, y0, za, zb);
    fused_tile<R, Src, Dst, TX, H>(g, src, dst, c, ring, fs.TY, x0, y0, za, zb, phi_in, rr);
}

template <typename R, typename Src, int TX>
__global__ __launch_bounds__(256, Occupancy<Src>::waves) void phase_tile_kernel(Geom g, Src src, R* __restrict__ phi,
                                                                               FusedShape fs) {
    extern __shared__ unsigned char lds_raw[];
    RecRing<TX> rr{reinterpret_cast<f4*>(lds_raw), fs.TY + 2};
    int x0, y0, za, zb;
    tile_of_block(fs, TX, g.nz, x0, y0, za, zb);
    phase_tile<R, Src, TX>(g, src, phi, rr, fs.TY, x0, y0, za, zb);
}

}  // namespace lbm
