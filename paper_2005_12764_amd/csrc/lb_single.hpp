// lb_single.hpp -- the one-read step: collide-and-stream tiles that also
// produce the phase-field sums of the next step.
//
// The phase field of a site is phi = D / Rc with D = sum_i d_i and
// Rc = sum_i (w_i + t_i) over its 19 pulled (post-streaming) populations.
// The collide pass writes those populations and holds them in registers, so
// each tile also sums, for every site of its own box, the terms whose source
// lies in the same box ("own" terms): a partial (D_own, Rc_own) per site.
// The terms whose source lies in another tile ("foreign": only sites on a
// face of their box have any) are pulled from the population arrays by a
// light assembly kernel that turns the partial sums of the face sites into
// phi; the tile writes phi of every other site itself.  Each
// population is read from HBM once per step (plus the few foreign ones),
// instead of once by a phase pass and again by the collide pass.
//
// The foreign terms that enter a site through an x face of its box all come
// from the one neighbouring tile column (a source that is also outside the
// y or z range of the box belongs to that face instead), so the tile holding
// those sources sums them per destination and stores the pair in a compact
// array after the own sums; the assembly reads one pair per x-face site
// instead of ten scattered values (rows are contiguous in x, so the y and z
// faces pull whole rows and keep the direct reads).
//
// Summation order is fixed, so results are reproducible: the own terms of a
// site in four groups -- sources in plane z-1, bounce-backs from the site
// itself, in-plane sources, sources in plane z+1 -- each in ascending
// direction; then the foreign terms of the z and the y faces, each in
// ascending direction; then the x-face sums (lo face, then hi face), each
// summed from zero in the group order of the own terms.  D and Rc are summed
// term by term alike, so a pure component (d_i = +-(w_i + t_i)) gives
// phi = +-1 exactly, as in the collision.
#pragma once
#include "lb_fused.hpp"

namespace lbm {

// Own partial sums of one site.
template <typename R>
struct Part2 {
    R dn, rc;
};

// A phase-sum buffer holds, for one state: the own sums of the sites on a
// face of their box (N pairs, indexed by site), the x-face sums of every tile
// column (2 faces x ny x nz pairs), and the phase field (N values).  The tile
// kernel writes phi itself for the sites whose every term is its own; the
// assembly completes the face sites.
template <int TX>
__host__ __device__ constexpr size_t xface_entries(int nx, int ny, int nz) {
    return (size_t)2 * ((nx + TX - 1) / TX) * ny * nz;
}
// Size of a phase-sum buffer in reals.
template <int TX>
__host__ __device__ constexpr size_t part_reals(int nx, int ny, int nz) {
    return 2 * ((size_t)nx * ny * nz + xface_entries<TX>(nx, ny, nz)) + (size_t)nx * ny * nz;
}
// The phase field of a phase-sum buffer.
template <int TX, typename R>
__host__ __device__ __forceinline__ R* phi_of(Part2<R>* part, const Geom& g) {
    return reinterpret_cast<R*>(part + (size_t)g.N + xface_entries<TX>(g.nx, g.ny, g.nz));
}

// Is the site a face site of its box (some source of its phase sums may lie
// in another box)?  x % TX, y % TY: position in the tile; za, zb: the chunk.
template <int TX, int TY>
__device__ __forceinline__ bool on_face(const Geom& g, int x, int y, int z, int za, int zb) {
    const int rx = x % TX, ry = y % TY;
    return rx == 0 || rx == TX - 1 || x == g.nx - 1 || ry == 0 || ry == TY - 1 || y == g.ny - 1 || z == za ||
           z == zb - 1;
}

// x-face sum of the site (x, y, z) on the lo (side 0, x = bx * TX) or hi
// (side 1) x face of tile column bx, in the compact array after the own sums.
__device__ __forceinline__ size_t xface_at(const Geom& g, int bx, int side, int y, int z) {
    return ((size_t)(bx * 2 + side) * g.nz + z) * g.ny + y;
}

// Direction with velocity (cx, cy, cz).
__host__ __device__ constexpr int dir_of(int cx, int cy, int cz) {
    for (int i = 0; i < Q; ++i)
        if (Lattice::cx[i] == cx && Lattice::cy[i] == cy && Lattice::cz[i] == cz) return i;
    return -1;
}

// Rows of the one-read tile (one site per thread and plane): 8, or 4 when
// the LDS of 8 rows exceeds the workgroup's budget (FP64 with a wide halo),
// or 16 (a 1024-thread workgroup, one per CU) when chosen by tile setting.
constexpr int kSingleTY = 8;
constexpr int kSingleTYSmall = 4;
constexpr int kSingleTYLarge = 16;

// Own box of a site: its tile column [x0, x1) x [y0, y1) and z chunk [z0, z1).
struct OwnBox {
    int x0, x1, y0, y1, z0, z1;
    __device__ __forceinline__ bool has(int x, int y, int z) const {
        return x >= x0 && x < x1 && y >= y0 && y < y1 && z >= z0 && z < z1;
    }
};

template <int TX, int TY>
__device__ __forceinline__ OwnBox box_of(const Geom& g, int TZ, int x, int y, int z) {
    OwnBox b;
    b.x0 = x - x % TX;
    b.x1 = min(b.x0 + TX, g.nx);
    b.y0 = y - y % TY;
    b.y1 = min(b.y0 + TY, g.ny);
    b.z0 = z - z % TZ;
    b.z1 = min(b.z0 + TZ, g.nz);
    return b;
}

// Group of direction i at a destination, in summation order: 0 = source in
// plane z-1, 1 = reflected from the site itself, 2 = in-plane source, 3 =
// source in plane z+1.
__device__ __forceinline__ int group_of(int i, bool reflected) {
    return reflected ? 1 : (Lattice::cz[i] > 0 ? 0 : (Lattice::cz[i] == 0 ? 2 : 3));
}

// Terms entering the site (x, y, z) with c_x = SX through its x face whose
// source lies within the y and z range of the site's box b, summed from zero
// in the group order of the own terms (sources in plane z-1, in-plane
// sources, sources in plane z+1), each group in ascending direction.
template <typename R, int SX, typename Src>
__device__ __forceinline__ Part2<R> xface_sum(const Geom& g, const Src& src, const OwnBox& b, int s, int x, int y,
                                             int z) {
    using L = Lattice;
    R dn = R(0), rc = R(0);
#pragma unroll
    for (int grp = 0; grp < 4; ++grp) {
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            if (L::cx[i] != SX || group_of(i, false) != grp) continue;
            const int ys = y - L::cy[i], zs = z - L::cz[i];
            if (ys < b.y0 || ys >= b.y1 || zs < b.z0 || zs >= b.z1) continue;
            int dir;
            const int sr = pull_source(g, i, x, y, z, s, dir);
            if (dir != i) continue;
            R t, d;
            src.template pull_one<R>(i, sr, dir, t, d);
            rc += weight<R>(i) + t;
            dn += d;
        }
    }
    return Part2<R>{dn, rc};
}

// Own partial sums (phi where they are complete) and x-face sums of the
// current state, for a state that no one-read step produced (initial,
// imported, or left by a two-pass step).
template <typename R, typename Src, int TX, int TY>
__global__ __launch_bounds__(256) void part_kernel(Geom g, Src src, int TZ, Part2<R>* __restrict__ part) {
    using L = Lattice;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.N) return;
    int x, y, z;
    site_xyz(g, s, x, y, z);
    const OwnBox b = box_of<TX, TY>(g, TZ, x, y, z);
    R dn = R(0), rc = R(0);
    R ph = R(0);  // own post-collision phase, for the moving-wall terms
    bool have_ph = false;
#pragma unroll
    for (int grp = 0; grp < 4; ++grp) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int dir;
            const int sr = pull_source(g, i, x, y, z, s, dir);
            const bool refl = dir != i;
            if (group_of(i, refl) != grp) continue;
            if (!refl && !b.has(x - L::cx[i], y - L::cy[i], z - L::cz[i])) continue;
            R t, d;
            src.template pull_one<R>(i, sr, dir, t, d);
            if constexpr (Src::moving) {
                // a reflection off a moving wall, as the pull adds it
                if (refl && g.moving) {
                    if (!have_ph) {
                        ph = src.template own_phase<R>(s);
                        have_ph = true;
                    }
                    const R add = wall_term<R>(g, i, x, y, z);
                    t += add;
                    d += add * ph;
                }
            }
            rc += weight<R>(i) + t;
            dn += d;
        }
    }
    if (on_face<TX, TY>(g, x, y, z, b.z0, b.z1)) part[s] = Part2<R>{dn, rc};
    else phi_of<TX>(part, g)[s] = dn / rc;
    // x-face sums of this site (beyond an x wall every term is a bounce-back)
    Part2<R>* xf = part + g.N;
    const bool lo = x % TX == 0 && !(g.wx && x == 0);
    const bool hi = (x % TX == TX - 1 || x == g.nx - 1) && !(g.wx && x == g.nx - 1);
    if (lo) xf[xface_at(g, x / TX, 0, y, z)] = xface_sum<R, 1>(g, src, b, s, x, y, z);
    if (hi) xf[xface_at(g, x / TX, 1, y, z)] = xface_sum<R, -1>(g, src, b, s, x, y, z);
}

// Walls next to a site: direction i arriving there is a bounce-back exactly
// when its upstream site lies beyond one of them (the test pull_source makes,
// without computing the upstream index).
struct WallFlags {
    bool xlo, xhi, ylo, yhi, zlo, zhi;
};
__device__ __forceinline__ WallFlags wall_flags(const Geom& g, int x, int y, int z) {
    return WallFlags{g.wx && x == 0, g.wx && x == g.nx - 1, g.wy && y == 0,
                     g.wy && y == g.ny - 1, g.wz && z == 0, g.wz && z == g.nz - 1};
}
__device__ __forceinline__ bool reflected(int i, const WallFlags& w) {
    using L = Lattice;
    return (L::cx[i] > 0 && w.xlo) || (L::cx[i] < 0 && w.xhi) || (L::cy[i] > 0 && w.ylo) ||
           (L::cy[i] < 0 && w.yhi) || (L::cz[i] > 0 && w.zlo) || (L::cz[i] < 0 && w.zhi);
}

// Faces of a site's own box along one axis: lo = first coordinate of its
// tile (sources at v - 1 lie outside), hi = last (sources at v + 1 outside).
struct Faces {
    bool lo, hi;
};
template <int T>
__device__ __forceinline__ Faces faces_of(int v, int n) {
    const int r = v % T;
    return Faces{r == 0, r == T - 1 || v == n - 1};
}
__device__ __forceinline__ Faces faces_z(int v, int z0, int z1) { return Faces{v == z0, v == z1 - 1}; }

// Does direction i leave the box through the faces f (c > 0 enters through
// lo, c < 0 through hi)?
__device__ __forceinline__ bool leaves(int c, const Faces& f) { return (c > 0 && f.lo) || (c < 0 && f.hi); }

// Foreign terms of site s = (x, y, z) whose source lies outside the box
// through the faces of `axis` (1 = y, 2 = z) and not through those of an
// axis summed before it (z, then y); bounce-backs are own terms.
template <typename R, typename Src, int AXIS>
__device__ __forceinline__ void foreign_terms(const Geom& g, const Src& src, int s, int x, int y, int z,
                                              const Faces& fy, const Faces& fz, R& dn, R& rc) {
    using L = Lattice;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const bool oz = leaves(L::cz[i], fz), oy = leaves(L::cy[i], fy);
        const bool mine = AXIS == 2 ? oz : (oy && !oz);
        if (!mine) continue;
        int dir;
        const int sr = pull_source(g, i, x, y, z, s, dir);
        if (dir != i) continue;
        R t, d;
        src.template pull_one<R>(i, sr, dir, t, d);
        rc += weight<R>(i) + t;
        dn += d;
    }
}

// Coordinates along an axis of extent n cut into boxes of T, ranked: the
// face coordinates (first and last of each box) and the inner ones.
struct AxisFaces {
    int n, T;
    __host__ __device__ int nface() const {
        if (T <= 2) return n;
        const int r = n % T;
        return 2 * (n / T) + (r == 0 ? 0 : (r == 1 ? 1 : 2));
    }
    __host__ __device__ int face(int k) const {
        if (T <= 2) return k;
        const int b = k >> 1, rest = n - b * T, size = rest < T ? rest : T;
        return b * T + ((k & 1) ? size - 1 : 0);
    }
    __host__ __device__ int inner(int m) const { return (m / (T - 2)) * T + m % (T - 2) + 1; }
};

// The face sites of the boxes, enumerated for the assembly: first every
// site of the face rows (the rows of a chunk's z faces, then the rows of a
// tile's y faces in the other planes), then the x-face sites of the
// remaining rows.
struct FaceSet {
    AxisFaces ax, ay, az;
    int nyf, nyi, nzf, nxf;
    int row_sites, edge_sites;
};
inline FaceSet face_set(const Geom& g, int TX, int TY, int TZ) {
    FaceSet f;
    f.ax = AxisFaces{g.nx, TX};
    f.ay = AxisFaces{g.ny, TY};
    f.az = AxisFaces{g.nz, TZ};
    f.nxf = f.ax.nface();
    f.nyf = f.ay.nface();
    f.nyi = g.ny - f.nyf;
    f.nzf = f.az.nface();
    const int nzi = g.nz - f.nzf;
    f.row_sites = (f.nzf * g.ny + nzi * f.nyf) * g.nx;
    f.edge_sites = nzi * f.nyi * f.nxf;
    return f;
}

// phi of the face sites from their own partial sums, the foreign terms of
// the z and y faces and the x-face sums.
template <typename R, typename Src, int TX, int TY>
__device__ __forceinline__ void assemble_site(const Geom& g, const Src& src, const FaceSet& fs,
                                              Part2<R>* __restrict__ part, int k) {
    int x, y, z;
    if (k < fs.row_sites) {
        const int r = k / g.nx, zrows = fs.nzf * g.ny;
        x = k - r * g.nx;
        if (r < zrows) {
            z = fs.az.face(r / g.ny);
            y = r - (r / g.ny) * g.ny;
        } else {
            const int r2 = r - zrows;
            z = fs.az.inner(r2 / fs.nyf);
            y = fs.ay.face(r2 - (r2 / fs.nyf) * fs.nyf);
        }
    } else {
        const int k2 = k - fs.row_sites;
        if (k2 >= fs.edge_sites) return;
        const int q = k2 / fs.nxf;
        x = fs.ax.face(k2 - q * fs.nxf);
        z = fs.az.inner(q / fs.nyi);
        y = fs.ay.inner(q - (q / fs.nyi) * fs.nyi);
    }
    const int s = site_of(g, x, y, z);
    const int TZ = fs.az.T, z0 = z - z % TZ;
    const Faces fx = faces_of<TX>(x, g.nx), fy = faces_of<TY>(y, g.ny), fz = faces_z(z, z0, min(z0 + TZ, g.nz));
    const Part2<R> P = part[s];
    R dn = P.dn, rc = P.rc;
    if (fz.lo || fz.hi) foreign_terms<R, Src, 2>(g, src, s, x, y, z, fy, fz, dn, rc);
    if (fy.lo || fy.hi) foreign_terms<R, Src, 1>(g, src, s, x, y, z, fy, fz, dn, rc);
    const Part2<R>* xf = part + g.N;
    if (fx.lo && !(g.wx && x == 0)) {
        const Part2<R> X = xf[xface_at(g, x / TX, 0, y, z)];
        dn += X.dn;
        rc += X.rc;
    }
    if (fx.hi && !(g.wx && x == g.nx - 1)) {
        const Part2<R> X = xf[xface_at(g, x / TX, 1, y, z)];
        dn += X.dn;
        rc += X.rc;
    }
    phi_of<TX>(part, g)[s] = dn / rc;
}

// Face site k of the enumeration above, one per thread.
template <typename R, typename Src, int TX, int TY>
__global__ __launch_bounds__(256) void assemble_kernel(Geom g, Src src, FaceSet fs, Part2<R>* __restrict__ part) {
    assemble_site<R, Src, TX, TY>(g, src, fs, part, blockIdx.x * blockDim.x + threadIdx.x);
}

// Exchange slot of a direction with c_y != 0 (the in-plane neighbours in
// other rows go through LDS; rows are wavefronts, so c_y = 0 neighbours are
// lane shuffles).
__host__ __device__ constexpr int xch_slot(int i) {
    return i == 3 ? 0 : i == 4 ? 1 : i == 7 ? 2 : i == 8 ? 3 : i == 9 ? 4 : i == 10 ? 5
         : i == 15 ? 6 : i == 16 ? 7 : i == 17 ? 8 : i == 18 ? 9 : -1;
}
constexpr int kXchDirs = 10;

template <typename R, int TX, int TY>
__host__ __device__ constexpr size_t xch_bytes() {
    return (size_t)2 * kXchDirs * TX * TY * sizeof(R);
}
// x-face sums an edge lane of a tile column accumulates for the face sites of
// the neighbouring column: the lo edge lane (SX = -1) feeds the hi face of
// the column on its left, the hi edge lane (SX = +1) the lo face of the one
// on its right (periodic wrap; none beyond an x wall).  The running sums of
// the destination planes z-1, z, z+1 of its row live in LDS, vs[side][plane
// mod 3][row].
template <int TX>
__device__ __forceinline__ bool xface_dest(const Geom& g, int x0, int x1, int SX, int& bd) {
    if (SX < 0) {
        if (x0 > 0) {
            bd = x0 / TX - 1;
            return true;
        }
        bd = (g.nx + TX - 1) / TX - 1;
        return !g.wx;
    }
    if (x1 < g.nx) {
        bd = x0 / TX + 1;
        return true;
    }
    bd = 0;
    return !g.wx;
}

// Before the exchange barrier: the lane's own terms of plane cz close the
// sum of destination plane cz - 1 (stored), add the first in-plane term of
// plane cz and open the sum of plane cz + 1.
template <typename R, int TY, int SX>
__device__ __forceinline__ void xedge_own(const Geom& g, const R (&t)[Q], const R (&d)[Q], Part2<R>* __restrict__ vs,
                                          int ty, int y, int cz, int za, int zb, int bd, Part2<R>* __restrict__ xf) {
    constexpr int im = dir_of(SX, 0, -1), i0 = dir_of(SX, 0, 0), ip = dir_of(SX, 0, 1);
    constexpr int side = SX < 0 ? 0 : 1;
    Part2<R>* v = vs + side * 3 * TY + ty;
    if (cz - 1 >= za) {
        Part2<R> P = v[((cz - 1 - za) % 3) * TY];
        P.rc += weight<R>(im) + t[im];
        P.dn += d[im];
        xf[xface_at(g, bd, 1 - side, y, cz - 1)] = P;
    }
    Part2<R> P = cz == za ? Part2<R>{R(0), R(0)} : v[((cz - za) % 3) * TY];
    P.rc += weight<R>(i0) + t[i0];
    P.dn += d[i0];
    v[((cz - za) % 3) * TY] = P;
    if (cz + 1 < zb) v[((cz + 1 - za) % 3) * TY] = Part2<R>{R(0) + d[ip], R(0) + (weight<R>(ip) + t[ip])};
}

// After the exchange barrier: the in-plane terms from the rows above and
// below (ascending direction); the chunk's last plane is then complete.
template <typename R, int TX, int TY, int SX>
__device__ __forceinline__ void xedge_rows(const Geom& g, const R* __restrict__ xch, Part2<R>* __restrict__ vs, int ty,
                                           int tx, int nrows, int y, int cz, int za, int zb, int bd,
                                           Part2<R>* __restrict__ xf) {
    using L = Lattice;
    constexpr int NT = TX * TY;
    constexpr int side = SX < 0 ? 0 : 1;
    Part2<R>* v = vs + side * 3 * TY + ty;
    Part2<R> P = v[((cz - za) % 3) * TY];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (L::cx[i] != SX || L::cz[i] != 0 || L::cy[i] == 0) continue;
        const int ys = ty - L::cy[i];
        if (ys < 0 || ys >= nrows) continue;
        P.rc += xch[(2 * xch_slot(i)) * NT + ys * TX + tx];
        P.dn += xch[(2 * xch_slot(i) + 1) * NT + ys * TX + tx];
    }
    if (cz == zb - 1) xf[xface_at(g, bd, 1 - side, y, cz)] = P;
    else v[((cz - za) % 3) * TY] = P;
}

// One tile of the one-read step: columns [x0, x0+TX) x [y0, y0+TY), planes
// [za, zb); blockDim.x == TX * TY and TX is the wavefront size.  Every thread
// of the workgroup must call it (it holds barriers).
template <typename R, typename Src, typename Dst, int TX, int TY, int H>
__device__ __forceinline__ void single_tile(const Geom& g, const Src& src, const Dst& dst, const Coeffs<R>& c,
                                            const PhiRing<R, TX, H>& ring, const RecRing<TX>& rr,
                                            R* __restrict__ xch, Part2<R>* __restrict__ vs, int x0, int y0,
                                            int za, int zb, const R* __restrict__ phi_in,
                                            Part2<R>* __restrict__ part_out, R* __restrict__ phi_out) {
    using L = Lattice;
    constexpr int LX = TX + 2 * H;
    constexpr int NP = 2 * H + 1;
    constexpr int NT = TX * TY;
    constexpr int LY = TY + 2 * H;
    const int tid = threadIdx.x;
    const int ty_ = tid / TX, tx_ = tid - (tid / TX) * TX;
    const int x_ = x0 + tx_, y_ = y0 + ty_;
    const bool active = x_ < g.nx && y_ < g.ny;
    const int x1 = min(x0 + TX, g.nx), y1 = min(y0 + TY, g.ny);
    // edge lanes and the columns their x-face sums go to
    Part2<R>* const xf = part_out + g.N;
    int bd_lo = 0, bd_hi = 0;
    const bool edge_lo = active && tx_ == 0 && xface_dest<TX>(g, x0, x1, -1, bd_lo);
    const bool edge_hi = active && x_ == x1 - 1 && xface_dest<TX>(g, x0, x1, 1, bd_hi);
    // own sums of the destination planes cz - 1 (prev), cz (cur)
    R prev_dn = R(0), prev_rc = R(0), cur_dn = R(0), cur_rc = R(0);

    for (int p = za - H; p < zb + H; ++p) {
        const int slot = (p - (za - H)) % NP;
        // ---- phase field of plane p on the tile and its halo
        {
            R* dstp = ring.plane(slot);
            const int zz = halo_coord(p, g.nz, g.wz);
            for (int q = tid; q < LY * LX; q += NT) {
                const int ly = q / LX, lx = q - ly * LX;
                const int xx = halo_coord(x0 - H + lx, g.nx, g.wx);
                const int yy = halo_coord(y0 - H + ly, g.ny, g.wy);
                dstp[q] = phi_in[site_of(g, xx, yy, zz)];
            }
        }
        if constexpr (Src::ring) {
            const int qr = p - H + 1;
            if (qr >= za - 1 && qr <= zb) load_rec_plane<Src, TX>(g, src, rr, (qr - za + 1) % 3, x0, y0, qr);
        }
        __syncthreads();
        const int cz = p - H;
        if (cz >= za) {
            // ---- collide (x, y, cz)
            R t[Q], d[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) t[i] = d[i] = R(0);
            if (active) {
                // the site's coordinates, re-read each plane: kept loop-invariant, the
                // compiler hoists every stencil address out of the z loop and runs out
                // of registers
                int x = x_, y = y_, tx = tx_, ty = ty_;
                asm volatile("" : "+v"(x), "+v"(y), "+v"(tx), "+v"(ty));
                const int s0 = (cz - (za - H)) % NP;
                const int sm = (s0 + NP - 1) % NP, sp = (s0 + 1) % NP;
                const int s = site_of(g, x, y, cz);
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
                dst.store_as_read(s, t, d, tot);
                // bounce-backs into this site: its own values, before the in-plane group
                const WallFlags wf = wall_flags(g, x, y, cz);
#pragma unroll
                for (int i = 1; i < Q; ++i) {
                    if (!reflected(i, wf)) continue;
                    cur_rc += weight<R>(i) + t[L::opp[i]];
                    cur_dn += d[L::opp[i]];
                }
            }
            // ---- hand the stored values to the destinations of this plane's
            // populations: other rows through LDS, the same row by shuffles
            R sh_t[Q], sh_d[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const R a = weight<R>(i) + t[i];
                if (L::cy[i] != 0) {
                    xch[(2 * xch_slot(i)) * NT + tid] = a;
                    xch[(2 * xch_slot(i) + 1) * NT + tid] = d[i];
                } else if (L::cx[i] > 0) {
                    sh_t[i] = __shfl_up(a, 1, TX);
                    sh_d[i] = __shfl_up(d[i], 1, TX);
                } else if (L::cx[i] < 0) {
                    sh_t[i] = __shfl_down(a, 1, TX);
                    sh_d[i] = __shfl_down(d[i], 1, TX);
                } else {
                    sh_t[i] = a;
                    sh_d[i] = d[i];
                }
            }
            if (edge_lo) xedge_own<R, TY, -1>(g, t, d, vs, ty_, y_, cz, za, zb, bd_lo, xf);
            if (edge_hi) xedge_own<R, TY, 1>(g, t, d, vs, ty_, y_, cz, za, zb, bd_hi, xf);
            __syncthreads();
            if (edge_lo) xedge_rows<R, TX, TY, -1>(g, xch, vs, ty_, tx_, y1 - y0, y_, cz, za, zb, bd_lo, xf);
            if (edge_hi) xedge_rows<R, TX, TY, 1>(g, xch, vs, ty_, tx_, y1 - y0, y_, cz, za, zb, bd_hi, xf);
            if (active) {
                int x = x_, y = y_, tx = tx_, ty = ty_;
                asm volatile("" : "+v"(x), "+v"(y), "+v"(tx), "+v"(ty));
                // a site on an x or y face of the box keeps its own sums for the assembly
                const bool face_xy =
                    tx == 0 || tx == TX - 1 || x == g.nx - 1 || ty == 0 || ty == TY - 1 || y == g.ny - 1;
                // value of direction i from the source (x - cx, y - cy) in plane cz
                auto from = [&](int i, R& va, R& vd) {
                    if (L::cy[i] != 0) {
                        const int at = (ty - L::cy[i]) * TX + tx - L::cx[i];
                        va = xch[(2 * xch_slot(i)) * NT + at];
                        vd = xch[(2 * xch_slot(i) + 1) * NT + at];
                    } else {
                        va = sh_t[i];
                        vd = sh_d[i];
                    }
                };
                auto in_tile = [&](int i) {
                    const int xs = x - L::cx[i], ys = y - L::cy[i];
                    return xs >= x0 && xs < x1 && ys >= y0 && ys < y1;
                };
                // destination cz - 1: sources in plane cz are its last group
                if (cz - 1 >= za) {
                    const WallFlags wm = wall_flags(g, x, y, cz - 1);
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        if (L::cz[i] != -1) continue;
                        if (reflected(i, wm) || !in_tile(i)) continue;
                        R va, vd;
                        from(i, va, vd);
                        prev_rc += va;
                        prev_dn += vd;
                    }
                    const int sm1 = site_of(g, x, y, cz - 1);
                    if (cz - 1 == za || face_xy) part_out[sm1] = Part2<R>{prev_dn, prev_rc};
                    else phi_out[sm1] = prev_dn / prev_rc;
                }
                // destination cz: in-plane sources
                const WallFlags w0 = wall_flags(g, x, y, cz);
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    if (L::cz[i] != 0) continue;
                    if (reflected(i, w0) || !in_tile(i)) continue;
                    R va, vd;
                    from(i, va, vd);
                    cur_rc += va;
                    cur_dn += vd;
                }
                // destination cz + 1: sources in plane cz are its first group
                R next_dn = R(0), next_rc = R(0);
                if (cz + 1 < zb) {
                    const WallFlags wp = wall_flags(g, x, y, cz + 1);
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        if (L::cz[i] != 1) continue;
                        if (reflected(i, wp) || !in_tile(i)) continue;
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
                if (cz == zb - 1) part_out[site_of(g, x, y, cz)] = Part2<R>{prev_dn, prev_rc};
            }
        }
        // no barrier here: the next staging overwrites ring and record slots
        // that only this plane's collide read, and every thread passed the
        // barrier after that collide before it gathers; the exchange buffer is
        // next written after the next staging's barrier
    }
}

template <typename R, typename Src, typename Dst, int TX, int TY, int H>
__global__ __launch_bounds__(TX * TY) void single_kernel(Geom g, Src src, Dst dst, Coeffs<R> c, FusedShape fs,
                                                        const Part2<R>* __restrict__ part_in,
                                                        Part2<R>* __restrict__ part_out) {
    extern __shared__ unsigned char lds_raw[];
    PhiRing<R, TX, H> ring{reinterpret_cast<R*>(lds_raw), TY + 2 * H};
    size_t off = (phi_ring_bytes<R, TX, H>(TY) + 15) & ~size_t(15);
    RecRing<TX> rr{reinterpret_cast<f4*>(lds_raw + off), TY + 2};
    if constexpr (Src::ring) off += rec_ring_bytes<TX>(TY);
    R* xch = reinterpret_cast<R*>(lds_raw + off);
    Part2<R>* vs = reinterpret_cast<Part2<R>*>(lds_raw + off + xch_bytes<R, TX, TY>());
    int x0, y0, za, zb;
    tile_of_block(fs, TX, g.nz, x0, y0, za, zb);
    single_tile<R, Src, Dst, TX, TY, H>(g, src, dst, c, ring, rr, xch, vs, x0, y0, za, zb,
                                        phi_of<TX>(const_cast<Part2<R>*>(part_in), g), part_out,
                                        phi_of<TX>(part_out, g));
}

}  // namespace lbm
