// d3q19.hpp -- device-side lattice tables and the local colour-gradient
// collision for gfx950.  Device code only; every loop over directions is
// fully unrolled so the lattice vectors and weights fold into immediates.
//
// Method (arXiv 2005.12764):
//   equilibrium w_i rho (1 + u_i + q_i)                     Sec. 2, eq:equil
//   BGK with mixture rate w_eff and harmonic nu_bar          Sec. 2.1, eq:twobgk
//   exact-difference source f^eq(u + F/rho) - f^eq(u)        Sec. 2.1, eq:edm
//   near-contact force F_rep = -A_h[h] n delta_I             Sec. 4
// plus the colour-gradient perturbation (Reis-Phillips, D3Q19 coefficients
// of Liu-Valocchi-Kang) and Latva-Kokko-Rothman recolouring, which the paper
// uses but does not write out.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int Q = 19;

// Direction order: rest, +x,-x,+y,-y,+z,-z, then the 12 face diagonals in
// opposite pairs.  This order is part of the library's state layout.
struct Lattice {
    static constexpr int cx[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int cz[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr int opp[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    static constexpr int len2(int i) { return cx[i] * cx[i] + cy[i] * cy[i] + cz[i] * cz[i]; }
};

template <typename R>
__host__ __device__ constexpr R weight(int i) {
    return Lattice::len2(i) == 0 ? R(1) / R(3) : (Lattice::len2(i) == 1 ? R(1) / R(18) : R(1) / R(36));
}
// B_i of the perturbation operator: -1/3, 1/18, 1/36 by shell.
template <typename R>
__host__ __device__ constexpr R bpert(int i) {
    return Lattice::len2(i) == 0 ? -R(1) / R(3) : (Lattice::len2(i) == 1 ? R(1) / R(18) : R(1) / R(36));
}
// 1/|c_i| (0 for the rest vector, whose recolouring term vanishes).
template <typename R>
__host__ __device__ constexpr R inv_clen(int i) {
    return Lattice::len2(i) == 0 ? R(0)
                                 : (Lattice::len2(i) == 1 ? R(1) : R(0.70710678118654752440084436210485));
}

// Per-lattice constants in the compute type, prepared on the host.
template <typename R>
struct Coeffs {
    R inv_nu_r, inv_nu_b;  // 1 / nu_k, nu_k = (tau_k - 1/2)/3
    R omega;               // the mixture rate when tau_r == tau_b (then 1/tau at every site)
    R half_A;              // A/2 of the perturbation
    R beta;
    R eps_g, eps_g2;       // |G| at or below which n = 0, and its square
    R g_iface, g_iface2;   // interface threshold of the near-contact probe, and its square
    R nc_strength, nc_hmin;
    R fx, fy, fz;          // body force density
    int nc_range;          // 0 = near-contact off
    int same_tau;          // tau_r == tau_b: omega above holds everywhere
    int model;             // 0 colour gradient, 1 Shan-Chen
    R g_sc;                // Shan-Chen coupling G_C
};

// c_i . a for a lattice velocity c_i (components -1, 0, 1): the sum of the
// non-zero components' terms only (a product by a zero component is not
// dropped by the compiler, since 0 * a is not 0 for every float a).
template <typename R>
__device__ __forceinline__ R cdot3(int i, R ax, R ay, R az) {
    using L = Lattice;
    R v = R(0);
    bool any = false;
    if (L::cx[i]) { v = L::cx[i] > 0 ? ax : -ax; any = true; }
    if (L::cy[i]) { const R b = L::cy[i] > 0 ? ay : -ay; v = any ? v + b : b; any = true; }
    if (L::cz[i]) { const R b = L::cz[i] > 0 ? az : -az; v = any ? v + b : b; }
    return v;
}

// Reciprocal and reciprocal square root.  FP32: the hardware estimates
// (v_rcp_f32, v_rsq_f32, within 1 ulp), used where an FP32 result only feeds
// further rounding-level arithmetic; FP64: correctly rounded.
__device__ __forceinline__ float rcp_of(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_of(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsq_of(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq_of(double x) { return 1.0 / sqrt(x); }

// Is |G| (G with squared length g2) above the threshold e (squared e2)?
// FP32 compares squares; FP64 compares the root, as the definition reads.
__device__ __forceinline__ bool above(float g2, float e, float e2) { (void)e; return g2 > e2; }
__device__ __forceinline__ bool above(double g2, double e, double e2) { (void)e2; return sqrt(g2) > e; }
__device__ __forceinline__ bool at_least(float g2, float e, float e2) { (void)e; return g2 >= e2; }
__device__ __forceinline__ bool at_least(double g2, double e, double e2) { (void)e2; return sqrt(g2) >= e; }
// 1/|G| for a G known to be non-zero.
__device__ __forceinline__ float inv_norm(float g2) { return rsq_of(g2); }
__device__ __forceinline__ double inv_norm(double g2) { return 1.0 / sqrt(g2); }

// Outputs of one site's collision that the 16-bit storage keeps per site.
template <typename R>
struct SiteTotals {
    R drho;                // post-collision density - 1
    R jx, jy, jz;          // 3 (j + F) = 3 rho v: the linear term of the equilibrium
    R phi;                 // phase x_r - x_b
    R vx, vy, vz;          // recolouring vector beta (rho_r rho_b/rho) G/|G|
};

// Local collision of one site, in shifted variables: t_i = f^r_i + f^b_i - w_i
// (the total's deviation from the rest equilibrium at unit density) and
// d_i = f^r_i - f^b_i (the colour difference).  Carrying the small t_i keeps
// FP32 rounding relative to the deviations that hold the flow, not to the
// O(w_i) populations (a per-step force increment is ~1e-7 of those).
// t/d hold the pulled (post-streaming) values on entry and the post-collision,
// recoloured values on exit.  (gx,gy,gz) is the colour gradient at the site,
// (Fx,Fy,Fz) the total force.  PAIRED: evaluate each direction together with
// its opposite (the same values up to rounding, fewer instructions: taken by
// the arithmetic-bound 16-bit tile; the memory-bound raw tiles measured
// faster with the per-direction form).
template <typename R, bool PAIRED = false>
__device__ __forceinline__ void collide(R (&t)[Q], R (&d)[Q], R gx, R gy, R gz, R Fx, R Fy, R Fz,
                                        const Coeffs<R>& c, SiteTotals<R>* tot = nullptr) {
    using L = Lattice;
    R drho = R(0), dif = R(0), rc = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        drho += t[i];
        dif += d[i];
        rc += weight<R>(i) + t[i];
        if (L::cx[i]) jx += L::cx[i] > 0 ? t[i] : -t[i];
        if (L::cy[i]) jy += L::cy[i] > 0 ? t[i] : -t[i];
        if (L::cz[i]) jz += L::cz[i] > 0 ? t[i] : -t[i];
    }
    const R rho = R(1) + drho;            // sum of the weights is 1
    // The colour split uses rc = sum_i (w_i + t_i), rounded term by term as
    // the colour difference is: a pure component (d_i = +-(w_i + t_i)) then
    // gives phi = +-1 exactly (a divided, not multiplied, quotient) and
    // x_r, x_b = 1, 0 exactly, and stays pure.
    const R phi = dif / rc;               // x_r - x_b
    const R xr = R(0.5) + R(0.5) * phi, xb = R(0.5) - R(0.5) * phi;
    const R inv_rho = rcp_of(rho);
    const R ux = jx * inv_rho, uy = jy * inv_rho, uz = jz * inv_rho;
    // exact-difference velocity shift du = F^k/rho_k with F^k = (rho_k/rho) F
    const R dx = Fx * inv_rho, dy = Fy * inv_rho, dz = Fz * inv_rho;
    const R vx = ux + dx, vy = uy + dy, vz = uz + dz;
    // s = u + (u + du): f^eq(u + du) - f^eq(u) = rho_k w_i [3 c.du + 4.5 (c.du)(c.s)
    // - 1.5 du.s], without subtracting two equilibria
    const R sx = ux + vx, sy = uy + vy, sz = uz + vz;
    const R ds = dx * sx + dy * sy + dz * sz;
    // mixture relaxation: 1/nu_bar = x_r/nu_r + x_b/nu_b, w = 2 cs2/(2 nu_bar + cs2)
    R omega = c.omega;
    if (!c.same_tau) {
        const R nubar = rcp_of(xr * c.inv_nu_r + xb * c.inv_nu_b);
        omega = R(2) * rcp_of(R(6) * nubar + R(1));
    }
    const R uu = ux * ux + uy * uy + uz * uz;

    const R g2 = gx * gx + gy * gy + gz * gz;
    const bool has_n = above(g2, c.eps_g, c.eps_g2);
    const R inv_gm = has_n ? inv_norm(g2) : R(0);
    const R gm = g2 * inv_gm;
    // perturbation amplitude (A/2)|G| and recolouring strength
    // beta rho_r rho_b / rho = beta x_r x_b rc
    const R pa = c.half_A * gm;
    const R seg = has_n ? c.beta * xr * xb * rc : R(0);
    const R nx = gx * inv_gm, ny = gy * inv_gm, nz = gz * inv_gm;

    if constexpr (PAIRED) {
        // rest direction (c = 0), then each pair (i, opposite): the even
        // terms once, the odd ones (c.u, c.du, c.n) with both signs
        {
            const R w0 = weight<R>(0);
            const R teq = w0 * (drho + rho * (-R(1.5) * uu));
            const R tp = t[0] - omega * (t[0] - teq) + rho * (w0 * (-R(1.5) * ds));
            const R ts = tp - pa * bpert<R>(0);
            t[0] = ts;
            d[0] = phi * (w0 + ts);
        }
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int o = L::opp[i];
            if (o < i) continue;  // evaluated with the first of the pair
            const R w = weight<R>(i);
            const R cu = cdot3<R>(i, ux, uy, uz);
            const R cd = cdot3<R>(i, dx, dy, dz);
            const R cs = cdot3<R>(i, sx, sy, sz);
            const R cn = cdot3<R>(i, nx, ny, nz);
            const R te = w * (drho + rho * (R(4.5) * cu * cu - R(1.5) * uu));  // teq, even part
            const R to = w * rho * (R(3) * cu);                               // teq, odd part
            const R se = rho * (w * (R(4.5) * cd * cs - R(1.5) * ds));        // rho * source, even
            const R so = rho * (w * (R(3) * cd));                             // rho * source, odd
            const R pert = pa * (w * cn * cn - bpert<R>(i));                  // perturbation (even)
            const R rec2 = R(2) * (seg * w * cn * inv_clen<R>(i));            // 2 rec (odd)
            const R tpi = t[i] - omega * (t[i] - (te + to)) + (se + so) + pert;
            const R tpo = t[o] - omega * (t[o] - (te - to)) + (se - so) + pert;
            t[i] = tpi;
            d[i] = phi * (w + tpi) + rec2;
            t[o] = tpo;
            d[o] = phi * (w + tpo) - rec2;
        }
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const R w = weight<R>(i);
            const R cu = cdot3<R>(i, ux, uy, uz);
            const R cd = cdot3<R>(i, dx, dy, dz);
            const R cs = cdot3<R>(i, sx, sy, sz);
            const R q = R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;                // f^eq/(w rho) - 1
            const R de = w * (R(3) * cd + R(4.5) * cd * cs - R(1.5) * ds);        // source / rho_k
            // total: BGK toward rho w (1 + q) (deviation w (drho + rho q)) plus rho de
            const R teq = w * (drho + rho * q);
            const R tp = t[i] - omega * (t[i] - teq) + rho * de;
            // (the components' own relaxation only enters through this total:
            // recolouring redistributes the colour from rho_r/rho and f*)
            const R cn = cdot3<R>(i, nx, ny, nz);   // c_i . n
            const R ts = tp + pa * (w * cn * cn - bpert<R>(i));                    // perturbation
            // recolouring: f^r = x_r f* + rec, f^b = x_b f* - rec, f* = w + t*
            const R rec = seg * w * cn * inv_clen<R>(i);
            t[i] = ts;
            d[i] = phi * (w + ts) + R(2) * rec;
        }
    }
    if (tot) {
        tot->drho = drho;
        tot->jx = R(3) * rho * vx;  // v = (j + F)/rho
        tot->jy = R(3) * rho * vy;
        tot->jz = R(3) * rho * vz;
        tot->phi = phi;
        tot->vx = seg * nx;
        tot->vy = seg * ny;
        tot->vz = seg * nz;
    }
}

// Local collision of one site in the Shan-Chen model (Sec. 2.1: the
// inter-component force of eq. shanchen_force entering each component's
// exact-difference source, eq:edm), in the shifted variables of collide().
// (bx,by,bz) = sum_i w_i rho_b(x + c_i) c_i and (rx,ry,rz) the same of rho_r.
// Component k gets the velocity shift du_k = F^k/rho_k with
// F^k = -G_C rho_k sum_i w_i rho_k'(x + c_i) c_i + (rho_k/rho) F_body, i.e.
// du_k = -G_C (that sum) + F_body/rho, with no division by rho_k; both relax
// with the mixture rate toward f^eq(rho_k, u), u = j/rho.  No perturbation
// and no recolouring: the force alone keeps the components apart.
template <typename R>
__device__ __forceinline__ void collide_sc(R (&t)[Q], R (&d)[Q], R bx, R by, R bz, R rx, R ry, R rz,
                                           const Coeffs<R>& c) {
    using L = Lattice;
    R drho = R(0), dif = R(0), rc = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        drho += t[i];
        dif += d[i];
        rc += weight<R>(i) + t[i];
        if (L::cx[i]) jx += L::cx[i] > 0 ? t[i] : -t[i];
        if (L::cy[i]) jy += L::cy[i] > 0 ? t[i] : -t[i];
        if (L::cz[i]) jz += L::cz[i] > 0 ? t[i] : -t[i];
    }
    const R rho = R(1) + drho;
    const R rr = R(0.5) * (rc + dif), rb = R(0.5) * (rc - dif);
    const R inv_rho = R(1) / rho;
    const R ux = jx * inv_rho, uy = jy * inv_rho, uz = jz * inv_rho;
    const R fx = c.fx * inv_rho, fy = c.fy * inv_rho, fz = c.fz * inv_rho;
    // velocity shifts of the red (R) and blue (B) components
    const R Rx = fx - c.g_sc * bx, Ry = fy - c.g_sc * by, Rz = fz - c.g_sc * bz;
    const R Bx = fx - c.g_sc * rx, By = fy - c.g_sc * ry, Bz = fz - c.g_sc * rz;
    // s_k = u + (u + du_k): f^eq(rho_k, u + du_k) - f^eq(rho_k, u)
    //   = rho_k w_i [3 c.du_k + 4.5 (c.du_k)(c.s_k) - 1.5 du_k.s_k]
    const R sRx = R(2) * ux + Rx, sRy = R(2) * uy + Ry, sRz = R(2) * uz + Rz;
    const R sBx = R(2) * ux + Bx, sBy = R(2) * uy + By, sBz = R(2) * uz + Bz;
    const R dsR = Rx * sRx + Ry * sRy + Rz * sRz;
    const R dsB = Bx * sBx + By * sBy + Bz * sBz;
    R omega = c.omega;
    if (!c.same_tau) {
        const R phi = dif / rc;
        const R xr = R(0.5) + R(0.5) * phi, xb = R(0.5) - R(0.5) * phi;
        const R nubar = R(1) / (xr * c.inv_nu_r + xb * c.inv_nu_b);
        omega = R(2) / (R(6) * nubar + R(1));
    }
    const R uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const R w = weight<R>(i);
        const R cu = cdot3<R>(i, ux, uy, uz);
        const R q = R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;
        const R teq = w * (drho + rho * q);          // f^eq(rho_r) + f^eq(rho_b) - w
        const R deq = w * dif * (R(1) + q);          // f^eq(rho_r) - f^eq(rho_b)
        const R cdR = cdot3<R>(i, Rx, Ry, Rz);
        const R csR = cdot3<R>(i, sRx, sRy, sRz);
        const R cdB = cdot3<R>(i, Bx, By, Bz);
        const R csB = cdot3<R>(i, sBx, sBy, sBz);
        const R SR = rr * w * (R(3) * cdR + R(4.5) * cdR * csR - R(1.5) * dsR);
        const R SB = rb * w * (R(3) * cdB + R(4.5) * cdB * csB - R(1.5) * dsB);
        t[i] = t[i] - omega * (t[i] - teq) + (SR + SB);
        d[i] = d[i] - omega * (d[i] - deq) + (SR - SB);
    }
}

// Shifted variables from the two components and back.
template <typename R>
__device__ __forceinline__ void to_shifted(int i, R fr, R fb, R& t, R& d) {
    t = (fr + fb) - weight<R>(i);
    d = fr - fb;
}
template <typename R>
__device__ __forceinline__ void from_shifted(int i, R t, R d, R& fr, R& fb) {
    const R f = weight<R>(i) + t;
    fr = R(0.5) * (f + d);
    fb = R(0.5) * (f - d);
}

// Equilibrium divided by the density, for the 16-bit codec and init.
template <typename R>
__device__ __forceinline__ R feq_unit(int i, R ux, R uy, R uz) {
    using L = Lattice;
    const R cu = cdot3<R>(i, ux, uy, uz);
    const R uu = ux * ux + uy * uy + uz * uz;
    return weight<R>(i) * (R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu);
}

// Near-contact amplitude A_h(h): full strength up to h_min, h^-3 beyond,
// zero outside 1..K.
template <typename R>
__device__ __forceinline__ R nc_amplitude(int h, const Coeffs<R>& c) {
    if (h < 1 || h > c.nc_range) return R(0);
    if (R(h) <= c.nc_hmin) return c.nc_strength;
    const R r = c.nc_hmin / R(h);
    return c.nc_strength * r * r * r;
}

}  // namespace lbm
