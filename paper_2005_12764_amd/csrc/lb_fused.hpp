// lb_fused.hpp -- single-pass colour-gradient step.
//
// A workgroup owns a tile of TX x TY columns and marches it through a chunk of
// z-planes.  For every plane entering the pipeline it pulls the populations of
// the tile plus a halo of H = K + 1 sites (K = near-contact range) and keeps
// only the phase field phi in an LDS ring of 2H+1 planes.  The plane H behind
// the newest one then has phi on every site its colour gradient, and the
// gradients along its near-contact probes, can reach: its interior sites pull
// their populations again (a recent read, served by the caches), collide and
// store.  Each site's populations cross HBM once per step in each direction;
// the halo and re-pulls are cache traffic.
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

// One tile: columns [x0, x0+TX) x [y0, y0+TY), planes [za, zb).  Every thread
// of the workgroup must call it (it holds barriers).
// phi_in == nullptr: the fused single pass computes phi from pulled
// populations; otherwise phi is read from the phase pass's array (collide
// pass of the two-pass step, z-marching with the same LDS ring).
template <typename R, typename Src, typename Dst, int TX, int H>
__device__ __forceinline__ void fused_tile(const Geom& g, const Src& src, const Dst& dst, const Coeffs<R>& c,
                                           const PhiRing<R, TX, H>& ring, int TY, int x0, int y0, int za,
                                           int zb, const R* __restrict__ phi_in = nullptr) {
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
                const int s = site_of(g, xx, yy, zz);
                if (phi_in) {
                    dstp[q] = phi_in[s];
                    continue;
                }
                R fr[Q], fb[Q];
                src.pull(g, s, xx, yy, zz, fr, fb);
                R rr = R(0), rb = R(0);
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    rr += fr[i];
                    rb += fb[i];
                }
                dstp[q] = (rr - rb) / (rr + rb);
            }
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
                R fr[Q], fb[Q];
                src.pull(g, s, x, y, cz, fr, fb);
                const int ly = ty + H, lx = tx + H;
                R gx, gy, gz;
                lds_gradient<R, TX, H>(ring, sm, s0, sp, ly, lx, gx, gy, gz);
                R Fx = c.fx, Fy = c.fy, Fz = c.fz;
                if (H > 1 && c.nc_range > 0) {
                    const R gm = sqrt(gx * gx + gy * gy + gz * gz);
                    if (gm >= c.g_iface) {
                        const R nx = -gx / gm, ny = -gy / gm, nz = -gz / gm;
                        int h = 0;
                        for (int k = 1; k <= c.nc_range && k < H; ++k) {
                            const int ox = (int)round(R(k) * nx);
                            const int oy = (int)round(R(k) * ny);
                            const int oz = (int)round(R(k) * nz);
                            // a probe sample beyond a wall ends the probe
                            if (g.wx && (x + ox < 0 || x + ox >= g.nx)) break;
                            if (g.wy && (y + oy < 0 || y + oy >= g.ny)) break;
                            if (g.wz && (cz + oz < 0 || cz + oz >= g.nz)) break;
                            const int t0 = (s0 + oz + NP) % NP;
                            R qx, qy, qz;
                            lds_gradient<R, TX, H>(ring, (t0 + NP - 1) % NP, t0, (t0 + 1) % NP, ly + oy,
                                                   lx + ox, qx, qy, qz);
                            const R qm = sqrt(qx * qx + qy * qy + qz * qz);
                            const R dot = qx * gx + qy * gy + qz * gz;
                            if (qm >= c.g_iface && dot < R(0)) {
                                h = k;
                                break;
                            }
                        }
                        const R ah = nc_amplitude<R>(h, c);
                        Fx += ah * gx;
                        Fy += ah * gy;
                        Fz += ah * gz;
                    }
                }
                SiteTotals<R> tot;
                collide<R>(fr, fb, gx, gy, gz, Fx, Fy, Fz, c, &tot);
                dst.store(s, fr, fb, tot);
            }
        }
        __syncthreads();
    }
}

template <typename R, typename Src, typename Dst, int TX, int H>
__global__ __launch_bounds__(256, (waves_of<Src, Dst>())) void fused_kernel(Geom g, Src src, Dst dst, Coeffs<R> c, FusedShape fs,
                                                    const R* __restrict__ phi_in) {
    extern __shared__ unsigned char lds_raw[];
    PhiRing<R, TX, H> ring{reinterpret_cast<R*>(lds_raw), fs.TY + 2 * H};
    // Workgroups are dealt round-robin to the 8 XCDs: give each XCD a
    // contiguous run of tiles so neighbouring tiles (which share halo rows)
    // run on the same L2.
    int b = blockIdx.x;
    if ((fs.nblocks & 7) == 0) b = (b & 7) * (fs.nblocks >> 3) + (b >> 3);
    const int tile = b % (fs.tiles_x * fs.tiles_y);
    const int chunk = b / (fs.tiles_x * fs.tiles_y);
    const int x0 = (tile % fs.tiles_x) * TX;
    const int y0 = (tile / fs.tiles_x) * fs.TY;
    const int za = chunk * fs.TZ;
    const int zb = min(za + fs.TZ, g.nz);
    fused_tile<R, Src, Dst, TX, H>(g, src, dst, c, ring, fs.TY, x0, y0, za, zb, phi_in);
}

}  // namespace lbm
