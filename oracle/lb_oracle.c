/*
 * lb_oracle.c -- plain FP64 CPU reference stepper for the two-component
 * colour-gradient lattice Boltzmann update on D3Q19.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  The GPU library never links, loads or
 * calls anything in here, and this file includes nothing from the library.
 *
 * It is deliberately slow and obvious: whole-lattice passes in the order the
 * method is stated, no blocking, no fusion, FP64 throughout, no fast-math.
 * OpenMP only splits the independent per-site loops across host threads; it
 * does not change any arithmetic.
 *
 * Method, by section of the paper (arXiv 2005.12764):
 *   - lattice update f_i(x+c_i,t+1) = (1-w) f_i + w f_i^eq + S_i     [Sec. 2, eq:eq1]
 *   - second-order equilibrium w_i rho (1 + u_i + q_i)                 [Sec. 2, eq:equil]
 *   - moments rho = sum f_i, u = sum f_i c_i / rho                      [Sec. 2, eq:eq2]
 *   - viscosity nu = c_s^2 (1/w - 1/2)                                  [Sec. 2, eq:eq3]
 *   - streaming is an exact memory shift                                 [Sec. 2, after eq:eq3]
 *   - two components r,b relaxing with one mixture rate w_eff, with the
 *     harmonic-mean mixture viscosity                                    [Sec. 2.1, eq:twobgk]
 *   - exact-difference-method source S = f^eq(u + F dt/rho) - f^eq(u)   [Sec. 2.1, eq:edm]
 *   - near-contact repulsion F_rep = -A_h[h] n delta_I                   [Sec. 4, F_rep equation]
 * The colour-gradient surface-tension perturbation and the recolouring step
 * are not written out in the paper; they follow the published colour-gradient
 * literature (Reis & Phillips 2007 perturbation in the D3Q19 form of Liu,
 * Valocchi & Kang 2012; Latva-Kokko & Rothman 2005 recolouring).
 *
 * Readings taken where the paper is silent or garbled (each is also listed
 * with the rest of the design notes):
 *   - w_eff = 2 c_s^2 / (2 nu_bar + c_s^2).  The printed form has a minus
 *     sign, which contradicts eq:eq3; the plus sign reduces to w = 1/tau.
 *   - the force on component k is (rho_k/rho) F, so both components receive
 *     the same velocity shift F/rho in the EDM source.
 *   - F_rep: delta_I = |G|, n = -G/|G| (outward normal), so F_rep = A_h G;
 *     h is the first k in 1..K at which the ray sample x + round(k n) is an
 *     interface site whose gradient opposes G(x).  The sampling is pinned by
 *     brute-force scans of films whose normal lies along a lattice axis, a
 *     face diagonal or the body diagonal; for other normals its parity is
 *     unpinned (checked only against the GPU path).
 *   - the colour gradient at a wall reads the mirror site across the
 *     halfway wall plane (neutral wetting).
 *
 * Storage: populations are f[k][i][site], k = 0 (red), 1 (blue), i = 0..18,
 * site = x + nx*(y + ny*z).  The state between steps is the post-streaming
 * (pre-collision) population set.
 *
 * Parameter vector prm[] (doubles):
 *   0 nx, 1 ny, 2 nz, 3..5 bc[x,y,z] (0 periodic, 1 halfway bounce-back walls),
 *   6 tau_r, 7 tau_b, 8 A (surface tension), 9 beta (recolouring),
 *   10 nc_strength, 11 nc_range K, 12 nc_hmin, 13..15 body force density,
 *   16 eps_g (|G| below which n = 0), 17 g_iface (interface threshold of the
 *   near-contact probe), 18..35 wall velocities of the six faces in the order
 *   -x, +x, -y, +y, -z, +z (3 components each; used on wall axes only),
 *   36 interface model (0 colour gradient, 1 Shan-Chen), 37 G_C (Shan-Chen
 *   coupling).
 *
 * Moving walls (the sheared channel of Sec. 5 has walls sliding at +-U): a
 * population reflected by a wall face moving with velocity U gains
 * 2 w_i rho_w (c_i . U)/c_s^2 with rho_w = 1, c_i its direction after the
 * reflection, shared between the components in the proportion rho_k/rho of
 * the reflecting site (its post-collision state), so a tangentially sliding
 * wall leaves every component's mass unchanged.  A population crossing two
 * wall faces (an edge) gets the sum of both faces' terms.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19

/* D3Q19: rest, 6 axis links, 12 face diagonals.  Opposite pairs are (1,2),
 * (3,4), ..., (17,18). */
static const int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

static double W[Q];      /* lattice weights */
static double BPERT[Q];  /* B_i of the perturbation operator */
static int tables_ready = 0;

static void init_tables(void) {
    if (tables_ready) return;
    for (int i = 0; i < Q; ++i) {
        int n2 = CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2];
        W[i] = (n2 == 0) ? 1.0 / 3.0 : (n2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
        BPERT[i] = (n2 == 0) ? -1.0 / 3.0 : (n2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
    }
    tables_ready = 1;
}

typedef struct {
    int n[3];
    int bc[3];
    double tau_r, tau_b, A, beta;
    double nc_strength;
    int nc_range;
    double nc_hmin;
    double force[3];
    double eps_g, g_iface;
    double uwall[6][3];
    int moving;
    int model;      /* 0 colour gradient, 1 Shan-Chen */
    double g_sc;    /* Shan-Chen coupling G_C */
} prm_t;

static prm_t unpack(const double *p) {
    prm_t q;
    for (int a = 0; a < 3; ++a) {
        q.n[a] = (int)p[a];
        q.bc[a] = (int)p[3 + a];
        q.force[a] = p[13 + a];
    }
    q.tau_r = p[6];
    q.tau_b = p[7];
    q.A = p[8];
    q.beta = p[9];
    q.nc_strength = p[10];
    q.nc_range = (int)p[11];
    q.nc_hmin = p[12];
    q.eps_g = p[16];
    q.g_iface = p[17];
    q.moving = 0;
    for (int f = 0; f < 6; ++f)
        for (int a = 0; a < 3; ++a) {
            q.uwall[f][a] = p[18 + 3 * f + a];
            if (q.uwall[f][a] != 0.0 && q.bc[f / 2]) q.moving = 1;
        }
    q.model = (int)p[36];
    q.g_sc = p[37];
    return q;
}

static size_t nsites(const prm_t *q) { return (size_t)q->n[0] * q->n[1] * q->n[2]; }

static size_t sidx(const prm_t *q, int x, int y, int z) {
    return (size_t)x + (size_t)q->n[0] * ((size_t)y + (size_t)q->n[1] * (size_t)z);
}

static void coords(const prm_t *q, size_t s, int *x, int *y, int *z) {
    *x = (int)(s % q->n[0]);
    *y = (int)((s / q->n[0]) % q->n[1]);
    *z = (int)(s / ((size_t)q->n[0] * q->n[1]));
}

/* Periodic wrap of a coordinate that may be off by any amount. */
static int wrap(int v, int n) {
    int r = v % n;
    return r < 0 ? r + n : r;
}

/* ------------------------------------------------------------------ */
/* Exported tables, for the table checks.                               */
/* ------------------------------------------------------------------ */
void orc_tables(int *c, double *w, int *opp, double *bpert) {
    init_tables();
    for (int i = 0; i < Q; ++i) {
        for (int a = 0; a < 3; ++a) c[3 * i + a] = CV[i][a];
        w[i] = W[i];
        opp[i] = OPP[i];
        bpert[i] = BPERT[i];
    }
}

/* ------------------------------------------------------------------ */
/* Equilibrium, Sec. 2 eq:equil with c_s^2 = 1/3:                       */
/*   f_i^eq = w_i rho (1 + c.u/cs2 + ((c.u)^2 - cs2 u^2)/(2 cs2^2))     */
/* ------------------------------------------------------------------ */
void orc_feq(double rho, const double *u, double *out) {
    init_tables();
    const double cs2 = 1.0 / 3.0;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
        out[i] = W[i] * rho * (1.0 + cu / cs2 + (cu * cu - cs2 * uu) / (2.0 * cs2 * cs2));
    }
}

/* Mixture relaxation rate, Sec. 2.1 eq:twobgk with the sign reading above.
 * nu_k = c_s^2 (tau_k - 1/2) from eq:eq3 with w_k = 1/tau_k. */
double orc_omega(double tau_r, double tau_b, double rho_r, double rho_b) {
    const double cs2 = 1.0 / 3.0;
    double nu_r = cs2 * (tau_r - 0.5);
    double nu_b = cs2 * (tau_b - 0.5);
    double rho = rho_r + rho_b;
    double inv_nu = (rho_r / rho) / nu_r + (rho_b / rho) / nu_b;
    double nubar = 1.0 / inv_nu;
    return 2.0 * cs2 / (2.0 * nubar + cs2);
}

/* BGK relaxation of one component toward f^eq(rho_k, u), plus the EDM
 * source f^eq(rho_k, u + du) - f^eq(rho_k, u)   [Sec. 2.1 eq:twobgk, eq:edm]. */
void orc_bgk_edm(double omega, double rho_k, const double *u, const double *du,
                 const double *fk, double *out) {
    double feq[Q], feq_s[Q], us[3];
    for (int a = 0; a < 3; ++a) us[a] = u[a] + du[a];
    orc_feq(rho_k, u, feq);
    orc_feq(rho_k, us, feq_s);
    for (int i = 0; i < Q; ++i)
        out[i] = (1.0 - omega) * fk[i] + omega * feq[i] + (feq_s[i] - feq[i]);
}

/* Colour-gradient surface-tension perturbation added to the total
 * population: (A/2)|G| [ w_i (c_i.G)^2/|G|^2 - B_i ]; zero when |G| <= eps. */
void orc_perturbation(double A, const double *G, double eps_g, double *out) {
    init_tables();
    double g = sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
    for (int i = 0; i < Q; ++i) {
        if (g <= eps_g) {
            out[i] = 0.0;
            continue;
        }
        double cg = CV[i][0] * G[0] + CV[i][1] * G[1] + CV[i][2] * G[2];
        out[i] = 0.5 * A * g * (W[i] * cg * cg / (g * g) - BPERT[i]);
    }
}

/* Recolouring (Latva-Kokko & Rothman): split the total post-collision
 * population f* into red and blue,
 *   f^r_i = (rho_r/rho) f*_i + beta (rho_r rho_b / rho) w_i cos(theta_i)
 *   f^b_i = (rho_b/rho) f*_i - beta (rho_r rho_b / rho) w_i cos(theta_i)
 * with cos(theta_i) = c_i.G / (|c_i| |G|), cos(theta_0) = 0, and no
 * anisotropic term when |G| <= eps. */
void orc_recolour(double rho_r, double rho_b, const double *fstar, const double *G,
                  double beta, double eps_g, double *out_r, double *out_b) {
    init_tables();
    double rho = rho_r + rho_b;
    double g = sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
    for (int i = 0; i < Q; ++i) {
        double cos_t = 0.0;
        if (i > 0 && g > eps_g) {
            double cl = sqrt((double)(CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2]));
            double cg = CV[i][0] * G[0] + CV[i][1] * G[1] + CV[i][2] * G[2];
            cos_t = cg / (cl * g);
        }
        double seg = beta * (rho_r * rho_b / rho) * W[i] * cos_t;
        out_r[i] = (rho_r / rho) * fstar[i] + seg;
        out_b[i] = (rho_b / rho) * fstar[i] - seg;
    }
}

/* Complete local collision at one site: moments, mixture rate, per-component
 * BGK + EDM with the force split F^k = (rho_k/rho) F, perturbation of the
 * total, recolouring.  G is the colour gradient at the site and F the total
 * force density acting on it. */
void orc_collide_site(const double *p, const double *fr, const double *fb, const double *G,
                      const double *F, double *out_r, double *out_b) {
    init_tables();
    prm_t q = unpack(p);
    double rho_r = 0.0, rho_b = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        rho_r += fr[i];
        rho_b += fb[i];
        for (int a = 0; a < 3; ++a) j[a] += (fr[i] + fb[i]) * CV[i][a];
    }
    double rho = rho_r + rho_b;
    double u[3], du[3];
    for (int a = 0; a < 3; ++a) {
        u[a] = j[a] / rho;
        du[a] = F[a] / rho; /* (F^k/rho_k) with F^k = (rho_k/rho) F */
    }
    double omega = orc_omega(q.tau_r, q.tau_b, rho_r, rho_b);
    double pr[Q], pb[Q], pert[Q], fstar[Q];
    orc_bgk_edm(omega, rho_r, u, du, fr, pr);
    orc_bgk_edm(omega, rho_b, u, du, fb, pb);
    orc_perturbation(q.A, G, q.eps_g, pert);
    for (int i = 0; i < Q; ++i) fstar[i] = pr[i] + pb[i] + pert[i];
    orc_recolour(rho_r, rho_b, fstar, G, q.beta, q.eps_g, out_r, out_b);
}

/* ------------------------------------------------------------------ */
/* Whole-lattice passes.                                                */
/* ------------------------------------------------------------------ */

/* Initial populations f^k_i = f^eq_i(rho_k, u); u may be NULL (zero). */
void orc_init(const double *p, const double *rho_r, const double *rho_b, const double *u,
              double *f) {
    init_tables();
    prm_t q = unpack(p);
    size_t N = nsites(&q);
#pragma omp parallel for schedule(static)
    for (long long s = 0; s < (long long)N; ++s) {
        double uu[3] = {0.0, 0.0, 0.0}, er[Q], eb[Q];
        if (u)
            for (int a = 0; a < 3; ++a) uu[a] = u[(size_t)a * N + s];
        orc_feq(rho_r[s], uu, er);
        orc_feq(rho_b[s], uu, eb);
        for (int i = 0; i < Q; ++i) {
            f[(size_t)i * N + s] = er[i];
            f[(size_t)(Q + i) * N + s] = eb[i];
        }
    }
}

/* Moments of the current (post-streaming) state, Sec. 2 eq:eq2:
 * rho_k = sum_i f^k_i, j = sum_i (f^r_i + f^b_i) c_i.  Any output may be NULL. */
void orc_moments(const double *p, const double *f, double *rho_r, double *rho_b, double *j) {
    init_tables();
    prm_t q = unpack(p);
    size_t N = nsites(&q);
#pragma omp parallel for schedule(static)
    for (long long s = 0; s < (long long)N; ++s) {
        double rr = 0.0, rb = 0.0, m[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i) {
            double a = f[(size_t)i * N + s], b = f[(size_t)(Q + i) * N + s];
            rr += a;
            rb += b;
            for (int d = 0; d < 3; ++d) m[d] += (a + b) * CV[i][d];
        }
        if (rho_r) rho_r[s] = rr;
        if (rho_b) rho_b[s] = rb;
        if (j)
            for (int d = 0; d < 3; ++d) j[(size_t)d * N + s] = m[d];
    }
}

/* Neighbour coordinate for the gradient stencil: periodic axes wrap; on a wall
 * axis a neighbour beyond the halfway wall is replaced by its mirror image,
 * which for a unit step is the edge site itself. */
static int stencil_coord(int v, int n, int wall) {
    if (!wall) return wrap(v, n);
    if (v < 0) return -1 - v;
    if (v >= n) return 2 * n - 1 - v;
    return v;
}

/* Colour gradient G(x) = (1/c_s^2) sum_i w_i phi(x + c_i) c_i. */
void orc_phase_gradient(const double *p, const double *phi, double *G) {
    init_tables();
    prm_t q = unpack(p);
    size_t N = nsites(&q);
#pragma omp parallel for schedule(static)
    for (long long s = 0; s < (long long)N; ++s) {
        int x, y, z;
        coords(&q, (size_t)s, &x, &y, &z);
        double g[3] = {0.0, 0.0, 0.0};
        for (int i = 1; i < Q; ++i) {
            int xn = stencil_coord(x + CV[i][0], q.n[0], q.bc[0]);
            int yn = stencil_coord(y + CV[i][1], q.n[1], q.bc[1]);
            int zn = stencil_coord(z + CV[i][2], q.n[2], q.bc[2]);
            double ph = phi[sidx(&q, xn, yn, zn)];
            for (int a = 0; a < 3; ++a) g[a] += W[i] * ph * CV[i][a];
        }
        for (int a = 0; a < 3; ++a) G[(size_t)a * N + s] = 3.0 * g[a];
    }
}

/* Near-contact strength A_h(h): the full strength up to h_min, then an h^-3
 * decay, zero beyond the probe range (Sec. 4, F_rep equation). */
double orc_nc_amplitude(double strength, double hmin, int K, int h) {
    if (h < 1 || h > K) return 0.0;
    if ((double)h <= hmin) return strength;
    double r = hmin / (double)h;
    return strength * r * r * r;
}

/* Near-contact repulsion F_rep = -A_h[h] n delta_I with n = -G/|G| and
 * delta_I = |G|, i.e. A_h G, at interface sites |G(x)| >= g_iface whose
 * outward ray x + round(k n), k = 1..K, meets an interface site with
 * G(y).G(x) < 0 first at k = h.  A ray sample beyond a wall ends the probe. */
void orc_nearcontact(const double *p, const double *G, double *Fnc) {
    init_tables();
    prm_t q = unpack(p);
    size_t N = nsites(&q);
#pragma omp parallel for schedule(static)
    for (long long s = 0; s < (long long)N; ++s) {
        double g[3], F[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 3; ++a) g[a] = G[(size_t)a * N + s];
        double gm = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        if (q.nc_strength != 0.0 && q.nc_range > 0 && gm >= q.g_iface) {
            int x0[3];
            coords(&q, (size_t)s, &x0[0], &x0[1], &x0[2]);
            int h = 0;
            for (int k = 1; k <= q.nc_range && h == 0; ++k) {
                int y[3], outside = 0;
                for (int a = 0; a < 3; ++a) {
                    double na = -g[a] / gm; /* outward unit normal */
                    int v = x0[a] + (int)round((double)k * na);
                    if (q.bc[a]) {
                        if (v < 0 || v >= q.n[a]) outside = 1;
                        y[a] = v;
                    } else {
                        y[a] = wrap(v, q.n[a]);
                    }
                }
                if (outside) break;
                size_t t = sidx(&q, y[0], y[1], y[2]);
                double gy[3];
                for (int a = 0; a < 3; ++a) gy[a] = G[(size_t)a * N + t];
                double gym = sqrt(gy[0] * gy[0] + gy[1] * gy[1] + gy[2] * gy[2]);
                double dot = gy[0] * g[0] + gy[1] * g[1] + gy[2] * g[2];
                if (gym >= q.g_iface && dot < 0.0) h = k;
            }
            double Ah = orc_nc_amplitude(q.nc_strength, q.nc_hmin, q.nc_range, h);
            for (int a = 0; a < 3; ++a) F[a] = Ah * g[a];
        }
        for (int a = 0; a < 3; ++a) Fnc[(size_t)a * N + s] = F[a];
    }
}

/* ------------------------------------------------------------------ */
/* Shan-Chen interface model (Sec. 2.1, "Multi-component flows").       */
/* ------------------------------------------------------------------ */

/* Inter-component force densities of eq. shanchen_force,
 *   F^r(x) = -G_C rho_r(x) sum_i w_i rho_b(x + c_i) c_i,
 *   F^b(x) = -G_C rho_b(x) sum_i w_i rho_r(x + c_i) c_i.
 * The paper states that positive G_C repels; its printed formula has no
 * minus sign, which would make positive G_C attract, so the sign is taken
 * from the statement (the usual Shan-Chen form).  A neighbour beyond a
 * halfway wall is its mirror image, as for the colour gradient.
 * rho_r, rho_b: N values; Fr, Fb: [3][N]. */
void orc_sc_force(const double *p, const double *rho_r, const double *rho_b, double *Fr, double *Fb) {
    init_tables();
    prm_t q = unpack(p);
    size_t N = nsites(&q);
#pragma omp parallel for schedule(static)
    for (long long s = 0; s < (long long)N; ++s) {
        int x, y, z;
        coords(&q, (size_t)s, &x, &y, &z);
        double sb[3] = {0.0, 0.0, 0.0}, sr[3] = {0.0, 0.0, 0.0};
        for (int i = 1; i < Q; ++i) {
            int xn = stencil_coord(x + CV[i][0], q.n[0], q.bc[0]);
            int yn = stencil_coord(y + CV[i][1], q.n[1], q.bc[1]);
            int zn = stencil_coord(z + CV[i][2], q.n[2], q.bc[2]);
            size_t t = sidx(&q, xn, yn, zn);
            for (int a = 0; a < 3; ++a) {
                sb[a] += W[i] * rho_b[t] * CV[i][a];
                sr[a] += W[i] * rho_r[t] * CV[i][a];
            }
        }
        for (int a = 0; a < 3; ++a) {
            Fr[(size_t)a * N + s] = -q.g_sc * rho_r[s] * sb[a];
            Fb[(size_t)a * N + s] = -q.g_sc * rho_b[s] * sr[a];
        }
    }
}

/* Local collision of one site in the Shan-Chen model: both components relax
 * with the mixture rate toward f^eq(rho_k, u), u = j/rho (Sec. 2.1,
 * eq:twobgk), each with its own exact-difference source
 * f^eq(rho_k, u + F^k/rho_k) - f^eq(rho_k, u) (eq:edm), where F^k is the
 * component's Shan-Chen force plus its share (rho_k/rho) of the body force.
 * No perturbation and no recolouring: the force alone keeps the components
 * apart.  A component absent from the site (rho_k = 0) has a zero source. */
void orc_sc_collide_site(const double *p, const double *fr, const double *fb, const double *Fr,
                         const double *Fb, double *out_r, double *out_b) {
    init_tables();
    prm_t q = unpack(p);
    double rho_r = 0.0, rho_b = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        rho_r += fr[i];
        rho_b += fb[i];
        for (int a = 0; a < 3; ++a) j[a] += (fr[i] + fb[i]) * CV[i][a];
    }
    double rho = rho_r + rho_b;
    double u[3], dur[3], dub[3];
    for (int a = 0; a < 3; ++a) {
        u[a] = j[a] / rho;
        double Fkr = Fr[a] + (rho_r / rho) * q.force[a];
        double Fkb = Fb[a] + (rho_b / rho) * q.force[a];
        dur[a] = rho_r > 0.0 ? Fkr / rho_r : 0.0;
        dub[a] = rho_b > 0.0 ? Fkb / rho_b : 0.0;
    }
    double omega = orc_omega(q.tau_r, q.tau_b, rho_r, rho_b);
    orc_bgk_edm(omega, rho_r, u, dur, fr, out_r);
    orc_bgk_edm(omega, rho_b, u, dub, fb, out_b);
}

/* Collision of the whole lattice: f (post-streaming) -> fpost (post-collision,
 * pre-streaming).  Optional outputs of the intermediate fields (NULL = skip):
 * phi[N], G[3N], Fnc[3N]; in the Shan-Chen model G receives F^r and Fnc
 * receives F^b. */
void orc_collide(const double *p, const double *f, double *fpost, double *phi_out,
                 double *G_out, double *Fnc_out) {
    init_tables();
    prm_t q = unpack(p);
    size_t N = nsites(&q);
    double *rr = (double *)malloc(N * sizeof(double));
    double *rb = (double *)malloc(N * sizeof(double));
    double *phi = (double *)malloc(N * sizeof(double));
    double *G = (double *)malloc(3 * N * sizeof(double));
    double *Fnc = (double *)malloc(3 * N * sizeof(double));

    /* 1. moments and the phase field phi = (rho_r - rho_b)/rho */
    orc_moments(p, f, rr, rb, NULL);
    for (size_t s = 0; s < N; ++s) phi[s] = (rr[s] - rb[s]) / (rr[s] + rb[s]);
    if (q.model == 1) {
        /* Shan-Chen: forces from the component densities, then the local
         * collision; G_out and Fnc_out receive F^r and F^b */
        orc_sc_force(p, rr, rb, G, Fnc);
#pragma omp parallel for schedule(static)
        for (long long s = 0; s < (long long)N; ++s) {
            double fr[Q], fb[Q], orr[Q], ob[Q], Fr[3], Fb[3];
            for (int i = 0; i < Q; ++i) {
                fr[i] = f[(size_t)i * N + s];
                fb[i] = f[(size_t)(Q + i) * N + s];
            }
            for (int a = 0; a < 3; ++a) {
                Fr[a] = G[(size_t)a * N + s];
                Fb[a] = Fnc[(size_t)a * N + s];
            }
            orc_sc_collide_site(p, fr, fb, Fr, Fb, orr, ob);
            for (int i = 0; i < Q; ++i) {
                fpost[(size_t)i * N + s] = orr[i];
                fpost[(size_t)(Q + i) * N + s] = ob[i];
            }
        }
        goto done;
    }
    /* 2. colour gradient */
    orc_phase_gradient(p, phi, G);
    /* 3. near-contact force */
    orc_nearcontact(p, G, Fnc);
    /* 4..8. local collision with F = F_body + F_rep */
#pragma omp parallel for schedule(static)
    for (long long s = 0; s < (long long)N; ++s) {
        double fr[Q], fb[Q], orr[Q], ob[Q], g[3], F[3];
        for (int i = 0; i < Q; ++i) {
            fr[i] = f[(size_t)i * N + s];
            fb[i] = f[(size_t)(Q + i) * N + s];
        }
        for (int a = 0; a < 3; ++a) {
            g[a] = G[(size_t)a * N + s];
            F[a] = q.force[a] + Fnc[(size_t)a * N + s];
        }
        orc_collide_site(p, fr, fb, g, F, orr, ob);
        for (int i = 0; i < Q; ++i) {
            fpost[(size_t)i * N + s] = orr[i];
            fpost[(size_t)(Q + i) * N + s] = ob[i];
        }
    }
done:
    if (phi_out) memcpy(phi_out, phi, N * sizeof(double));
    if (G_out) memcpy(G_out, G, 3 * N * sizeof(double));
    if (Fnc_out) memcpy(Fnc_out, Fnc, 3 * N * sizeof(double));
    free(rr);
    free(rb);
    free(phi);
    free(G);
    free(Fnc);
}

/* Streaming: f^k_i(x + c_i) <- fpost^k_i(x).  A population whose target lies
 * beyond a wall on any wall axis is reflected back to its own site into the
 * opposite direction (halfway bounce-back), plus the moving-wall term of every
 * wall face it crosses; periodic axes wrap. */
void orc_stream(const double *p, const double *fpost, double *f) {
    init_tables();
    prm_t q = unpack(p);
    size_t N = nsites(&q);
#pragma omp parallel for schedule(static)
    for (long long s = 0; s < (long long)N; ++s) {
        int x0[3];
        coords(&q, (size_t)s, &x0[0], &x0[1], &x0[2]);
        double xr = 0.0; /* red fraction of the site, for moving-wall terms */
        if (q.moving) {
            double a = 0.0, b = 0.0;
            for (int i = 0; i < Q; ++i) {
                a += fpost[(size_t)i * N + s];
                b += fpost[(size_t)(Q + i) * N + s];
            }
            xr = a / (a + b);
        }
        for (int i = 0; i < Q; ++i) {
            int y[3], blocked = 0;
            double cu = 0.0; /* c_opp(i) . U summed over the crossed faces */
            for (int a = 0; a < 3; ++a) {
                int v = x0[a] + CV[i][a];
                if (q.bc[a] && (v < 0 || v >= q.n[a])) {
                    blocked = 1;
                    const double *U = q.uwall[2 * a + (v < 0 ? 0 : 1)];
                    for (int b = 0; b < 3; ++b) cu += CV[OPP[i]][b] * U[b];
                }
                y[a] = wrap(v, q.n[a]);
            }
            if (blocked) {
                double fr = fpost[(size_t)i * N + s], fb = fpost[(size_t)(Q + i) * N + s];
                double add = 2.0 * W[OPP[i]] * cu / (1.0 / 3.0); /* rho_w = 1 */
                f[(size_t)OPP[i] * N + s] = fr + add * xr;
                f[(size_t)(Q + OPP[i]) * N + s] = fb + add * (1.0 - xr);
            } else {
                for (int k = 0; k < 2; ++k)
                    f[(size_t)(k * Q + i) * N + sidx(&q, y[0], y[1], y[2])] = fpost[(size_t)(k * Q + i) * N + s];
            }
        }
    }
}

/* n full steps (collide, then stream).  f_in and f_out may be the same. */
void orc_step(const double *p, const double *f_in, double *f_out, int nsteps) {
    prm_t q = unpack(p);
    size_t M = 2 * Q * nsites(&q);
    double *cur = (double *)malloc(M * sizeof(double));
    double *post = (double *)malloc(M * sizeof(double));
    memcpy(cur, f_in, M * sizeof(double));
    for (int t = 0; t < nsteps; ++t) {
        orc_collide(p, cur, post, NULL, NULL, NULL);
        orc_stream(p, post, cur);
    }
    memcpy(f_out, cur, M * sizeof(double));
    free(cur);
    free(post);
}

/* ---------------------------------------------------------------------------
 * Korteweg-tensor diagnostic of the coarse-graining pipeline (Sec. 4.1, the
 * Korteweg tensor in terms of the Laplacian and the gradient products of the
 * field, and the projection by block averages).  The field is the phase field
 * phi of the state; derivatives use the same D3Q19 stencils and the same
 * mirror rule at walls as the colour gradient.
 * ------------------------------------------------------------------------- */

/* Phase field phi = (rho_r - rho_b)/(rho_r + rho_b) of the post-streaming
 * state (Sec. 2, the colour-gradient model's order parameter). */
void orc_phase_field(const double *p, const double *f, double *phi) {
    init_tables();
    prm_t q = unpack(p);
    size_t N = nsites(&q);
#pragma omp parallel for schedule(static)
    for (long long s = 0; s < (long long)N; ++s) {
        double rr = 0.0, rb = 0.0;
        for (int i = 0; i < Q; ++i) {
            rr += f[(size_t)i * N + s];
            rb += f[(size_t)(Q + i) * N + s];
        }
        phi[s] = (rr - rb) / (rr + rb);
    }
}

/* K_ab = lam [phi Lap(phi) + |grad phi|^2 / 2] delta_ab - lam d_a phi d_b phi
 * at every site, with grad phi = (1/c_s^2) sum_i w_i c_i phi(x + c_i) and
 * Lap(phi) = (2/c_s^2) sum_i w_i [phi(x + c_i) - phi(x)].  K is [6][N] in the
 * order xx, yy, zz, xy, xz, yz. */
void orc_korteweg(const double *p, const double *phi, double lam, double *K) {
    init_tables();
    prm_t q = unpack(p);
    size_t N = nsites(&q);
#pragma omp parallel for schedule(static)
    for (long long s = 0; s < (long long)N; ++s) {
        int x, y, z;
        coords(&q, (size_t)s, &x, &y, &z);
        double g[3] = {0.0, 0.0, 0.0}, lap = 0.0;
        for (int i = 1; i < Q; ++i) {
            int xn = stencil_coord(x + CV[i][0], q.n[0], q.bc[0]);
            int yn = stencil_coord(y + CV[i][1], q.n[1], q.bc[1]);
            int zn = stencil_coord(z + CV[i][2], q.n[2], q.bc[2]);
            double ph = phi[sidx(&q, xn, yn, zn)];
            for (int a = 0; a < 3; ++a) g[a] += W[i] * ph * CV[i][a];
            lap += W[i] * (ph - phi[s]);
        }
        for (int a = 0; a < 3; ++a) g[a] *= 3.0;
        lap *= 6.0;
        double iso = lam * (phi[s] * lap + 0.5 * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]));
        K[0 * N + s] = iso - lam * g[0] * g[0];
        K[1 * N + s] = iso - lam * g[1] * g[1];
        K[2 * N + s] = iso - lam * g[2] * g[2];
        K[3 * N + s] = -lam * g[0] * g[1];
        K[4 * N + s] = -lam * g[0] * g[2];
        K[5 * N + s] = -lam * g[1] * g[2];
    }
}

/* Projection of ncomp fields [ncomp][N] onto blocks of b x b x b sites
 * (Sec. 4.1, averaging over blocks): out[c][zc][yc][xc] is the mean over the
 * block's sites.  Every extent must be a multiple of b. */
void orc_block_average(const double *p, const double *field, int ncomp, int b, double *out) {
    prm_t q = unpack(p);
    size_t N = nsites(&q);
    int nxc = q.n[0] / b, nyc = q.n[1] / b, nzc = q.n[2] / b;
    size_t Nc = (size_t)nxc * nyc * nzc;
    for (int c = 0; c < ncomp; ++c)
        for (int zc = 0; zc < nzc; ++zc)
            for (int yc = 0; yc < nyc; ++yc)
                for (int xc = 0; xc < nxc; ++xc) {
                    double sum = 0.0;
                    for (int k = 0; k < b; ++k)
                        for (int j = 0; j < b; ++j)
                            for (int i = 0; i < b; ++i)
                                sum += field[(size_t)c * N + sidx(&q, xc * b + i, yc * b + j, zc * b + k)];
                    out[(size_t)c * Nc + ((size_t)zc * nyc + yc) * nxc + xc] = sum / ((double)b * b * b);
                }
}

/* Number of host threads the parallel loops use (1 without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
int orc_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int n) { omp_set_num_threads(n); }
#else
int orc_threads(void) { return 1; }
void orc_set_threads(int n) { (void)n; }
#endif
