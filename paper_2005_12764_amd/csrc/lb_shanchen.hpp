// lb_shanchen.hpp -- the two passes of a step in the Shan-Chen interface
// model (Sec. 2.1, "Multi-component flows": the inter-component force of
// eq. shanchen_force with the exact-difference source of eq:edm), for raw
// (FP64/FP32) storage.
//
// Density pass: the component densities (rho_r, rho_b) of every site of the
// current (post-streaming) state, as pairs.  Collide pass: 64-wide tiles
// marching a z-chunk with the density pairs of planes z-1, z, z+1 (tile plus
// one site) in an LDS ring; every site pulls its 19 populations per
// component, takes the two stencil sums sum_i w_i rho_k(x + c_i) c_i from the
// ring (mirror images beyond walls), collides (collide_sc) and stores.
#pragma once
#include "lb_fused.hpp"

namespace lbm {

template <typename R>
struct RhoPair {
    R r, b;
};

template <typename R, typename Src>
__global__ __launch_bounds__(256) void sc_density_kernel(Geom g, Src src, RhoPair<R>* __restrict__ rho2) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.N) return;
    int x, y, z;
    site_xyz(g, s, x, y, z);
    R t[Q], d[Q];
    src.pull(g, s, x, y, z, t, d);
    R rc = R(0), dif = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        rc += weight<R>(i) + t[i];
        dif += d[i];
    }
    rho2[s] = RhoPair<R>{R(0.5) * (rc + dif), R(0.5) * (rc - dif)};
}

template <typename R>
__host__ __device__ constexpr size_t sc_ring_bytes(int TY, int TX) {
    return (size_t)3 * (TY + 2) * (TX + 2) * sizeof(RhoPair<R>);
}

template <typename R, typename Src, typename Dst, int TX>
__global__ __launch_bounds__(256) void sc_collide_kernel(Geom g, Src src, Dst dst, Coeffs<R> c, FusedShape fs,
                                                         const RhoPair<R>* __restrict__ rho2) {
    using L = Lattice;
    extern __shared__ unsigned char lds_raw[];
    RhoPair<R>* ring = reinterpret_cast<RhoPair<R>*>(lds_raw);
    constexpr int LX = TX + 2;
    const int TY = fs.TY, LY = TY + 2;
    const int tid = threadIdx.x, nt = blockDim.x;
    int x0, y0, za, zb;
    tile_of_block(fs, TX, g.nz, x0, y0, za, zb);
    for (int p = za - 1; p <= zb; ++p) {
        const int slot = (p - (za - 1)) % 3;
        {
            RhoPair<R>* dstp = ring + (size_t)slot * LY * LX;
            const int zz = halo_coord(p, g.nz, g.wz);
            for (int q = tid; q < LY * LX; q += nt) {
                const int ly = q / LX, lx = q - ly * LX;
                const int xx = halo_coord(x0 - 1 + lx, g.nx, g.wx);
                const int yy = halo_coord(y0 - 1 + ly, g.ny, g.wy);
                dstp[q] = rho2[site_of(g, xx, yy, zz)];
            }
        }
        __syncthreads();
        const int cz = p - 1;
        if (cz >= za) {
            const RhoPair<R>* pl[3] = {ring + (size_t)((cz - 1 - (za - 1)) % 3) * LY * LX,
                                       ring + (size_t)((cz - (za - 1)) % 3) * LY * LX,
                                       ring + (size_t)((cz + 1 - (za - 1)) % 3) * LY * LX};
            for (int q = tid; q < TY * TX; q += nt) {
                const int ty = q / TX, tx = q - ty * TX;
                const int x = x0 + tx, y = y0 + ty;
                if (x >= g.nx || y >= g.ny) continue;
                const int s = site_of(g, x, y, cz);
                R t[Q], d[Q];
                src.pull(g, s, x, y, cz, t, d);
                R bx = R(0), by = R(0), bz = R(0), rx = R(0), ry = R(0), rz = R(0);
#pragma unroll
                for (int i = 1; i < Q; ++i) {
                    const RhoPair<R> v = pl[1 + L::cz[i]][(ty + 1 + L::cy[i]) * LX + tx + 1 + L::cx[i]];
                    const R wb = weight<R>(i) * v.b, wr = weight<R>(i) * v.r;
                    if (L::cx[i]) { bx += L::cx[i] > 0 ? wb : -wb; rx += L::cx[i] > 0 ? wr : -wr; }
                    if (L::cy[i]) { by += L::cy[i] > 0 ? wb : -wb; ry += L::cy[i] > 0 ? wr : -wr; }
                    if (L::cz[i]) { bz += L::cz[i] > 0 ? wb : -wb; rz += L::cz[i] > 0 ? wr : -wr; }
                }
                collide_sc<R>(t, d, bx, by, bz, rx, ry, rz, c);
                dst.store(s, t, d, SiteTotals<R>{});
            }
        }
        __syncthreads();
    }
}

}  // namespace lbm
