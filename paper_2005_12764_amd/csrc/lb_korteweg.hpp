// lb_korteweg.hpp -- Korteweg-tensor diagnostic of the phase field, projected
// on blocks (the coarse-graining data of Sec. 4.1).
//
// K_ab = lam [phi Lap(phi) + |grad phi|^2 / 2] delta_ab - lam d_a phi d_b phi
// with the D3Q19 stencils grad phi = 3 sum_i w_i c_i phi(x + c_i) and
// Lap(phi) = 6 sum_i w_i (phi(x + c_i) - phi(x)) (mirror sites beyond walls,
// as for the colour gradient), averaged with phi over blocks of b x b x b
// sites.
//
// One workgroup covers 64 columns x 8 rows and marches a chunk of planes
// (a one-dimensional grid of tiles x chunks, mapped to XCDs in runs),
// the phase field of four planes (tile plus a one-site halo) in an LDS ring,
// so each value is read from HBM about once.  Each thread sums its column's
// seven values over the b planes of a block layer; at the end of a layer the
// lanes combine the b columns of a block by a butterfly of shuffles and the
// first wavefront adds the block's b rows in order, so every result is
// reproducible.
#pragma once
#include "lb_kernels.hpp"

namespace lbm {

constexpr int kKortewegRows = 8;    // rows of a workgroup (a multiple of every b)
constexpr int kKortewegChunk = 32;  // planes a workgroup marches (a multiple of every b)

template <typename R, typename Out>
__global__ __launch_bounds__(64 * kKortewegRows) void korteweg_kernel(Geom g, const R* __restrict__ phi, R lam,
                                                                      int b, Out* __restrict__ kout,
                                                                      Out* __restrict__ pout, int accumulate) {
    using L = Lattice;
    constexpr int TY = kKortewegRows, LX = 64 + 2, LY = TY + 2, NP = 4;
    __shared__ R ring[NP * LY * LX];
    __shared__ R acc[TY * 64 * 7];  // [row][block column][value]
    const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
    // tile of this workgroup: workgroups are dealt round-robin to the 8 XCDs,
    // so the map gives each XCD a contiguous run of tiles (x fastest, then y,
    // then chunks); neighbouring tiles then share their halo rows and columns
    // in one L2 instead of fetching them from HBM twice
    const int tx = (g.nx + 63) / 64, tyn = (g.ny + TY - 1) / TY;
    const int nb = (int)gridDim.x;
    int blk = (int)blockIdx.x;
    if ((nb & 7) == 0) blk = (blk & 7) * (nb >> 3) + (blk >> 3);
    const int tile = blk % (tx * tyn), chunk = blk / (tx * tyn);
    const int x0 = (tile % tx) * 64, y0 = (tile / tx) * TY, za = chunk * kKortewegChunk;
    const int zb = min(za + kKortewegChunk, g.nz);
    const int x = x0 + lane, y = y0 + row;
    const bool active = x < g.nx && y < g.ny;
    const int cols = 64 / b;
    R sum[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) sum[c] = R(0);
    // the staged window: the tile plus a one-site halo, LY x LX values per
    // plane; each thread stages the entries q = threadIdx.x + k * 512
    constexpr int NT = 64 * TY, PER = (LY * LX + NT - 1) / NT;
    auto load_plane = [&](int p, R (&v)[PER]) {
        const int zz = stencil_coord(p, g.nz, g.wz);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int q = threadIdx.x + k * NT;
            if (q < LY * LX) {
                const int ly = q / LX, lx = q - ly * LX;
                // coordinates past the first one beyond the lattice only feed
                // inactive threads: clamp them into the stencil's range
                const int xx = stencil_coord(min(x0 - 1 + lx, g.nx), g.nx, g.wx);
                const int yy = stencil_coord(min(y0 - 1 + ly, g.ny), g.ny, g.wy);
                v[k] = phi[site_of(g, xx, yy, zz)];
            }
        }
    };
    auto store_plane = [&](int p, const R (&v)[PER]) {
        R* dst = ring + ((p + NP) % NP) * (LY * LX);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int q = threadIdx.x + k * NT;
            if (q < LY * LX) dst[q] = v[k];
        }
    };
    R nxt[PER];
    load_plane(za - 1, nxt);
    store_plane(za - 1, nxt);
    load_plane(za, nxt);
    store_plane(za, nxt);
    load_plane(za + 1, nxt);
    for (int z = za; z < zb; ++z) {
        // LDS holds planes z-1 and z; plane z+1 arrives from registers, and
        // the loads of plane z+2 are in flight while plane z is computed
        store_plane(z + 1, nxt);
        __syncthreads();
        if (z + 2 <= zb) load_plane(z + 2, nxt);
        // K at (x, y, z) from planes z-1, z, z+1
        if (active) {
            const R* pm = ring + ((z - 1 + NP) % NP) * (LY * LX);
            const R* p0 = ring + ((z + NP) % NP) * (LY * LX);
            const R* pp = ring + ((z + 1 + NP) % NP) * (LY * LX);
            const int c0 = (row + 1) * LX + lane + 1;
            const R f0 = p0[c0];
            R gx = R(0), gy = R(0), gz = R(0), lap = R(0);
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const R* pl = L::cz[i] > 0 ? pp : (L::cz[i] < 0 ? pm : p0);
                const R pn = pl[c0 + L::cy[i] * LX + L::cx[i]];
                const R wp = weight<R>(i) * pn;
                if (L::cx[i]) gx += L::cx[i] > 0 ? wp : -wp;
                if (L::cy[i]) gy += L::cy[i] > 0 ? wp : -wp;
                if (L::cz[i]) gz += L::cz[i] > 0 ? wp : -wp;
                lap += weight<R>(i) * (pn - f0);
            }
            gx *= R(3);
            gy *= R(3);
            gz *= R(3);
            lap *= R(6);
            const R iso = lam * (f0 * lap + R(0.5) * (gx * gx + gy * gy + gz * gz));
            sum[0] += iso - lam * gx * gx;
            sum[1] += iso - lam * gy * gy;
            sum[2] += iso - lam * gz * gz;
            sum[3] += -lam * gx * gy;
            sum[4] += -lam * gx * gz;
            sum[5] += -lam * gy * gz;
            sum[6] += f0;
        }
        if ((z - za) % b != b - 1) continue;
        // a block layer is complete: the b columns, then the b rows of each block
        for (int m = 1; m < b; m <<= 1) {
#pragma unroll
            for (int c = 0; c < 7; ++c) sum[c] += __shfl_xor(sum[c], m, 64);
        }
        if (lane % b == 0) {
#pragma unroll
            for (int c = 0; c < 7; ++c) acc[(row * cols + lane / b) * 7 + c] = sum[c];
        }
#pragma unroll
        for (int c = 0; c < 7; ++c) sum[c] = R(0);
        __syncthreads();
        if (threadIdx.x < cols * (TY / b)) {
            const int bc = threadIdx.x % cols, br = threadIdx.x / cols;  // block column, block row
            const int nxc = g.nx / b, nyc = g.ny / b;
            const int xc = x0 / b + bc, yc = y0 / b + br, zc = z / b;
            if (xc < nxc && yc < nyc) {
                const size_t Nc = (size_t)nxc * nyc * (g.nz / b);
                const size_t at = ((size_t)zc * nyc + yc) * nxc + xc;
                const R inv = R(1) / R(b * b * b);
#pragma unroll
                for (int c = 0; c < 7; ++c) {
                    R v = R(0);
                    for (int r = 0; r < b; ++r) v += acc[((br * b + r) * cols + bc) * 7 + c];
                    v *= inv;
                    Out* o = c < 6 ? (kout ? kout + c * Nc + at : nullptr) : (pout ? pout + at : nullptr);
                    if (o) *o = accumulate ? Out(*o + Out(v)) : Out(v);
                }
            }
        }
    }
}

}  // namespace lbm
