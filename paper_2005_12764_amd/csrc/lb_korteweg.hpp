// lb_korteweg.hpp -- Korteweg-tensor diagnostic of the phase field, projected
// on blocks (the coarse-graining data of Sec. 4.1).
//
// K_ab = lam [phi Lap(phi) + |grad phi|^2 / 2] delta_ab - lam d_a phi d_b phi
// with the D3Q19 stencils grad phi = 3 sum_i w_i c_i phi(x + c_i) and
// Lap(phi) = 6 sum_i w_i (phi(x + c_i) - phi(x)) (mirror sites beyond walls,
// as for the colour gradient), averaged with phi over blocks of b x b x b
// sites.  One workgroup covers 64 columns x b rows of one block layer: each
// thread sums its site's seven values over the b planes of the layer, lanes
// combine across the b columns of a block by a butterfly of shuffles, and the
// first wavefront adds the b rows in order, so every result is reproducible.
#pragma once
#include "lb_kernels.hpp"

namespace lbm {

constexpr int kKortewegMaxB = 8;

template <typename R, typename Out>
__global__ __launch_bounds__(64 * kKortewegMaxB) void korteweg_kernel(Geom g, const R* __restrict__ phi, R lam,
                                                                      int b, Out* __restrict__ kout,
                                                                      Out* __restrict__ pout, int accumulate) {
    using L = Lattice;
    __shared__ R acc[64 * 7];  // [row][block column][value]: b rows x 64/b block columns
    const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
    const int x = blockIdx.x * 64 + lane, y = blockIdx.y * b + row;
    R sum[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) sum[c] = R(0);
    if (x < g.nx) {
        for (int z = blockIdx.z * b; z < blockIdx.z * b + b; ++z) {
            const R p0 = phi[site_of(g, x, y, z)];
            R gx = R(0), gy = R(0), gz = R(0), lap = R(0);
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int xn = L::cx[i] ? stencil_coord(x + L::cx[i], g.nx, g.wx) : x;
                const int yn = L::cy[i] ? stencil_coord(y + L::cy[i], g.ny, g.wy) : y;
                const int zn = L::cz[i] ? stencil_coord(z + L::cz[i], g.nz, g.wz) : z;
                const R pn = phi[site_of(g, xn, yn, zn)];
                const R wp = weight<R>(i) * pn;
                if (L::cx[i]) gx += L::cx[i] > 0 ? wp : -wp;
                if (L::cy[i]) gy += L::cy[i] > 0 ? wp : -wp;
                if (L::cz[i]) gz += L::cz[i] > 0 ? wp : -wp;
                lap += weight<R>(i) * (pn - p0);
            }
            gx *= R(3);
            gy *= R(3);
            gz *= R(3);
            lap *= R(6);
            const R iso = lam * (p0 * lap + R(0.5) * (gx * gx + gy * gy + gz * gz));
            sum[0] += iso - lam * gx * gx;
            sum[1] += iso - lam * gy * gy;
            sum[2] += iso - lam * gz * gz;
            sum[3] += -lam * gx * gy;
            sum[4] += -lam * gx * gz;
            sum[5] += -lam * gy * gz;
            sum[6] += p0;
        }
    }
    // the b columns of a block: butterfly over lanes that differ in the low bits
    for (int m = 1; m < b; m <<= 1) {
#pragma unroll
        for (int c = 0; c < 7; ++c) sum[c] += __shfl_xor(sum[c], m, 64);
    }
    const int cols = 64 / b;
    if (lane % b == 0) {
#pragma unroll
        for (int c = 0; c < 7; ++c) acc[(row * cols + lane / b) * 7 + c] = sum[c];
    }
    __syncthreads();
    if (row == 0 && lane < cols) {
        const int nxc = g.nx / b, nyc = g.ny / b;
        const int xc = blockIdx.x * cols + lane;
        if (xc < nxc) {
            const size_t Nc = (size_t)nxc * nyc * (g.nz / b);
            const size_t at = ((size_t)blockIdx.z * nyc + blockIdx.y) * nxc + xc;
            const R inv = R(1) / R(b * b * b);
#pragma unroll
            for (int c = 0; c < 7; ++c) {
                R v = R(0);
                for (int r = 0; r < b; ++r) v += acc[(r * cols + lane) * 7 + c];
                v *= inv;
                Out* o = c < 6 ? (kout ? kout + c * Nc + at : nullptr) : (pout ? pout + at : nullptr);
                if (o) *o = accumulate ? Out(*o + Out(v)) : Out(v);
            }
        }
    }
}

}  // namespace lbm
