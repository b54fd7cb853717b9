// lb_api.hip -- host side of liblb.so: handle, parameter validation, buffer
// ownership, kernel dispatch and the C ABI declared in include/lb.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "lb.h"
#include "lb_internal.hpp"

using namespace lbm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return LB_OK;
    return fail(e == hipErrorOutOfMemory ? LB_ENOMEM : LB_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

namespace lbm {

int set_error(int code, const char* msg) { return fail(code, msg); }

int validate_params(const lb_params* p, std::string& why) {
    if (!p) return why = "params is NULL", LB_EINVAL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return why = "lattice sizes must be >= 1", LB_EINVAL;
    const double n = double(p->nx) * double(p->ny) * double(p->nz);
    if (n * Q > 9.0e18 || n >= 2147483647.0) return why = "lattice too large (sites must fit in 31 bits)", LB_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (p->bc[a] != 0 && p->bc[a] != 1) return why = "bc must be 0 (periodic) or 1 (walls)", LB_EINVAL;
    if (p->storage < LB_STORE_F64 || p->storage > LB_STORE_BF16) return why = "unknown storage", LB_EINVAL;
    if (p->kernel < LB_KERNEL_AUTO || p->kernel > LB_KERNEL_FUSED) return why = "unknown kernel", LB_EINVAL;
    if (!(p->tau_r > 0.5) || !(p->tau_b > 0.5) || !std::isfinite(p->tau_r) || !std::isfinite(p->tau_b))
        return why = "tau_r and tau_b must be finite and > 1/2", LB_EINVAL;
    if (!(p->A >= 0.0) || !std::isfinite(p->A)) return why = "A must be finite and >= 0", LB_EINVAL;
    if (!(p->beta >= 0.0 && p->beta <= 1.0)) return why = "beta must lie in [0, 1]", LB_EINVAL;
    if (!std::isfinite(p->nc_strength) || p->nc_strength < 0.0) return why = "nc_strength must be finite and >= 0", LB_EINVAL;
    if (p->nc_range < 0 || p->nc_range > LB_MAX_NC_RANGE) return why = "nc_range outside 0..LB_MAX_NC_RANGE", LB_EINVAL;
    if (!(p->nc_hmin > 0.0) && p->nc_range > 0 && p->nc_strength > 0) return why = "nc_hmin must be > 0", LB_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p->body_force[a])) return why = "body_force must be finite", LB_EINVAL;
    for (int f = 0; f < 6; ++f)
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(p->wall_velocity[f][a])) return why = "wall_velocity must be finite", LB_EINVAL;
    if (p->scale_log2 < 0 || p->scale_log2 > 24) return why = "scale_log2 outside 0..24", LB_EINVAL;
    if (!std::isfinite(p->eps_g) || !std::isfinite(p->g_iface)) return why = "eps_g, g_iface must be finite", LB_EINVAL;
    if (p->model != LB_MODEL_COLOUR_GRADIENT && p->model != LB_MODEL_SHAN_CHEN)
        return why = "unknown interface model", LB_EINVAL;
    if (p->model == LB_MODEL_SHAN_CHEN) {
        if (!std::isfinite(p->g_sc)) return why = "g_sc must be finite", LB_EINVAL;
        // the 16-bit codec stores the colour part in the form recolouring gives
        if (p->storage != LB_STORE_F64 && p->storage != LB_STORE_F32)
            return why = "the Shan-Chen model needs raw storage (LB_STORE_F64 or LB_STORE_F32)", LB_EINVAL;
        if (p->kernel == LB_KERNEL_FUSED)
            return why = "the Shan-Chen model steps with two passes (LB_KERNEL_AUTO or LB_KERNEL_TWOPASS)", LB_EINVAL;
    }
    return LB_OK;
}

template <typename R>
Coeffs<R> make_coeffs(const lb_params& p) {
    Coeffs<R> c;
    const double nu_r = (p.tau_r - 0.5) / 3.0, nu_b = (p.tau_b - 0.5) / 3.0;
    c.inv_nu_r = R(1.0 / nu_r);
    c.inv_nu_b = R(1.0 / nu_b);
    c.same_tau = p.tau_r == p.tau_b;
    c.omega = R(1.0 / p.tau_r);  // 2 cs2 / (2 nu + cs2) = 1/tau
    c.half_A = R(0.5 * p.A);
    c.beta = R(p.beta);
    const double eps = p.eps_g > 0 ? p.eps_g : (p.storage == LB_STORE_F64 ? 1e-12 : 1e-6);
    const double gi = p.g_iface > 0 ? p.g_iface : 0.05;
    c.eps_g = R(eps);
    c.eps_g2 = R(eps * eps);
    c.g_iface = R(gi);
    c.g_iface2 = R(gi * gi);
    c.nc_strength = R(p.nc_strength);
    c.nc_hmin = R(p.nc_hmin);
    c.fx = R(p.body_force[0]);
    c.fy = R(p.body_force[1]);
    c.fz = R(p.body_force[2]);
    c.nc_range = (p.nc_strength > 0.0 && p.model == LB_MODEL_COLOUR_GRADIENT) ? p.nc_range : 0;
    c.model = p.model;
    c.g_sc = R(p.g_sc);
    return c;
}
template Coeffs<double> make_coeffs<double>(const lb_params&);
template Coeffs<float> make_coeffs<float>(const lb_params&);

Geom make_geom(const lb_params& p) {
    Geom g;
    g.nx = p.nx;
    g.ny = p.ny;
    g.nz = p.nz;
    g.wx = p.bc[0];
    g.wy = p.bc[1];
    g.wz = p.bc[2];
    g.nxy = p.nx * p.ny;
    g.N = p.nx * p.ny * p.nz;
    g.moving = 0;
    for (int f = 0; f < 6; ++f)
        for (int a = 0; a < 3; ++a) {
            g.uw[f][a] = p.wall_velocity[f][a];
            if (p.wall_velocity[f][a] != 0.0 && p.bc[f / 2]) g.moving = 1;
        }
    return g;
}

size_t pop_bytes(int storage, size_t N) {
    switch (storage) {
        case LB_STORE_F64: return 2 * Q * raw_stride(N) * sizeof(double);
        case LB_STORE_F32: return 2 * Q * raw_stride(N) * sizeof(float);
        default: return 8 * N * sizeof(float) + Q * dev_stride(N) * 2;
    }
}

}  // namespace lbm

// ---------------------------------------------------------------------------
// Handle
// ---------------------------------------------------------------------------
struct lb_t {
    lb_params p;
    Geom g;
    hipStream_t stream;
    int device;
    void* buf[2];      // post-collision populations, ping-pong
    void* pending;     // raw FP32 state of a 16-bit lattice before its first step
    void* phi;         // phase field of the two-pass step (double for F64, float otherwise)
    void* part[2];     // phase sums and phase field of the one-read step, ping-pong
    int part_cur;      // part[part_cur] belongs to the current state ...
    bool part_valid;   // ... when this is set
    int part_ty = 0, part_tz = 0;  // tile boxes those sums follow
    Neu* partial;      // reduction partials
    double* dtot;      // device totals [14]
    int cur;           // buffer holding the current state
    int64_t steps;
    bool initialised;
    bool fresh;        // the state was set (init/import), no collision since: no wall terms
    int kernel;        // LB_KERNEL_TWOPASS or LB_KERNEL_FUSED
    Coeffs<double> cd;
    Coeffs<float> cf;
};

namespace {

lbm::LatticeView view_of(lb_t* h) {
    lbm::LatticeView v;
    v.p = &h->p;
    v.g = h->g;
    if (h->fresh) v.g.moving = 0;
    v.stream = h->stream;
    v.cur = h->buf[h->cur];
    v.nxt = h->buf[h->cur ^ 1];
    v.pending = h->pending;
    v.phi = h->phi;
    v.part_in = h->part[h->part_cur];
    v.part_out = h->part[h->part_cur ^ 1];
    // sums gathered for other tile boxes than the next step's are summed again
    if (h->part_valid) {
        const lbm::FusedShape fs = lbm::tile_shape(h->p, lbm::TILE_SINGLE);
        v.part_valid = fs.TY == h->part_ty && fs.TZ == h->part_tz;
    } else {
        v.part_valid = false;
    }
    v.cd = h->cd;
    v.cf = h->cf;
    return v;
}

void release(lb_t* h) {
    if (!h) return;
    if (h->buf[0]) (void)hipFree(h->buf[0]);
    if (h->buf[1]) (void)hipFree(h->buf[1]);
    if (h->pending) (void)hipFree(h->pending);
    if (h->phi) (void)hipFree(h->phi);
    if (h->part[0]) (void)hipFree(h->part[0]);
    if (h->part[1]) (void)hipFree(h->part[1]);
    if (h->partial) (void)hipFree(h->partial);
    if (h->dtot) (void)hipFree(h->dtot);
    delete h;
}

int copy_in(const void* src, int on_device, size_t bytes, void** dev_out, void* scratch, hipStream_t st) {
    if (on_device) {
        *dev_out = const_cast<void*>(src);
        return LB_OK;
    }
    int rc = check_hip(hipMemcpyAsync(scratch, src, bytes, hipMemcpyHostToDevice, st), "hipMemcpyAsync H2D");
    *dev_out = scratch;
    return rc;
}

}  // namespace

extern "C" {

const char* lb_last_error(void) { return g_err.c_str(); }

int lb_set_tiles(int32_t kind, int32_t storage, int32_t ty, int32_t tz) {
    static const int kind_of[4] = {TILE_PHASE, TILE_COLLIDE, TILE_SINGLE, TILE_BATCH};
    if (kind < LB_TILES_PHASE || kind > LB_TILES_BATCH) return fail(LB_EINVAL, "unknown tile kind");
    if (storage < LB_STORE_F64 || storage > LB_STORE_BF16) return fail(LB_EINVAL, "unknown storage");
    const bool rows_ok = kind == LB_TILES_ONE_READ ? (ty == 0 || ty == 4 || ty == 8 || ty == 16)
                                                   : (ty == 0 || ty == 1 || ty == 2 || ty == 4 || ty == 8 || ty == 16);
    if (!rows_ok || (kind == LB_TILES_BATCH && ty == 16)) return fail(LB_EINVAL, "tile rows not supported for this kind");
    if (tz < 0 || tz > 4096) return fail(LB_EINVAL, "tile planes outside 0..4096");
    set_tile_setting(kind_of[kind], storage, ty, tz);
    return LB_OK;
}

int64_t lb_footprint_bytes(const lb_params* p) {
    std::string why;
    if (validate_params(p, why) != LB_OK) return -1;
    const size_t N = size_t(p->nx) * p->ny * p->nz;
    const size_t real = p->storage == LB_STORE_F64 ? 8 : 4;
    size_t b = 2 * pop_bytes(p->storage, N) + N * real * (p->model == LB_MODEL_SHAN_CHEN ? 2 : 1);
    // phase sums of the one-read step (unless two passes are asked for; an
    // upper bound for lattices the automatic choice steps otherwise)
    if (p->kernel != LB_KERNEL_TWOPASS && p->model == LB_MODEL_COLOUR_GRADIENT)
        b += 2 * part_reals<kTX>(p->nx, p->ny, p->nz) * real;
    // a 16-bit lattice's raw FP32 initial state, kept from lb_init_fields
    if (p->storage >= LB_STORE_F16) b += pop_bytes(LB_STORE_F32, N);
    return (int64_t)b;
}

int lb_create(const lb_params* params, void* hip_stream, lb_t** out) {
    if (!out) return fail(LB_EINVAL, "out is NULL");
    *out = nullptr;
    std::string why;
    if (validate_params(params, why) != LB_OK) return fail(LB_EINVAL, why);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(LB_EDEVICE, "no HIP device");
    lb_t* h = new (std::nothrow) lb_t();
    if (!h) return fail(LB_ENOMEM, "host allocation failed");
    h->p = *params;
    if (h->p.scale_log2 == 0) h->p.scale_log2 = 16;
    h->g = make_geom(h->p);
    h->stream = (hipStream_t)hip_stream;
    (void)hipGetDevice(&h->device);
    h->cd = make_coeffs<double>(h->p);
    h->cf = make_coeffs<float>(h->p);
    h->kernel = choose_kernel(h->p);
    if (h->kernel < 0) {
        delete h;
        return fail(LB_EINVAL, "the fused kernel cannot hold this near-contact halo in LDS; use LB_KERNEL_TWOPASS");
    }
    const size_t N = (size_t)h->g.N;
    const size_t pb = pop_bytes(h->p.storage, N);
    int rc = LB_OK;
    if ((rc = check_hip(hipMalloc(&h->buf[0], pb), "hipMalloc populations")) ||
        (rc = check_hip(hipMalloc(&h->buf[1], pb), "hipMalloc populations")) ||
        (rc = check_hip(hipMalloc(&h->phi, N * (h->p.storage == LB_STORE_F64 ? 8 : 4) *
                                               (h->p.model == LB_MODEL_SHAN_CHEN ? 2 : 1)),
                        "hipMalloc phase field")) ||
        (rc = check_hip(hipMalloc((void**)&h->partial, sizeof(Neu) * NTOT * kTotalsBlocks), "hipMalloc partials")) ||
        (rc = check_hip(hipMalloc((void**)&h->dtot, sizeof(double) * 2 * NTOT), "hipMalloc totals"))) {
        release(h);
        return rc;
    }
    if (h->kernel == LB_KERNEL_FUSED) {
        const size_t pbytes = part_reals<kTX>(h->p.nx, h->p.ny, h->p.nz) * (h->p.storage == LB_STORE_F64 ? 8 : 4);
        if ((rc = check_hip(hipMalloc(&h->part[0], pbytes), "hipMalloc phase sums")) ||
            (rc = check_hip(hipMalloc(&h->part[1], pbytes), "hipMalloc phase sums"))) {
            release(h);
            return rc;
        }
    }
    *out = h;
    return LB_OK;
}

int lb_destroy(lb_t* h) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    (void)hipStreamSynchronize(h->stream);
    release(h);
    return LB_OK;
}

int lb_init_fields(lb_t* h, const void* rho_r, const void* rho_b, const void* u, int32_t dtype,
                   int32_t on_device) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (!rho_r || !rho_b) return fail(LB_EINVAL, "rho_r and rho_b are required");
    if (dtype != LB_DTYPE_F64 && dtype != LB_DTYPE_F32) return fail(LB_EINVAL, "dtype must be LB_DTYPE_F64 or LB_DTYPE_F32");
    const size_t N = (size_t)h->g.N;
    const size_t es = dtype == LB_DTYPE_F64 ? 8 : 4;
    if (!on_device) {
        // host inputs: reject non-physical densities before touching the state
        for (size_t s = 0; s < N; ++s) {
            const double a = dtype == LB_DTYPE_F64 ? ((const double*)rho_r)[s] : ((const float*)rho_r)[s];
            const double b = dtype == LB_DTYPE_F64 ? ((const double*)rho_b)[s] : ((const float*)rho_b)[s];
            if (!(a >= 0.0) || !(b >= 0.0) || !(a + b > 0.0) || !std::isfinite(a + b))
                return fail(LB_EINVAL, "densities must be finite, >= 0, with rho_r + rho_b > 0");
        }
    }
    // 16-bit lattices keep the initial state raw (FP32) until their first step.
    const bool split = h->p.storage >= LB_STORE_F16;
    if (split && !h->pending) {
        int rc = check_hip(hipMalloc(&h->pending, pop_bytes(LB_STORE_F32, N)), "hipMalloc initial state");
        if (rc) return rc;
    }
    void *d_rr = nullptr, *d_rb = nullptr, *d_u = nullptr, *scratch = nullptr;
    if (!on_device) {
        int rc = check_hip(hipMalloc(&scratch, 5 * N * es), "hipMalloc staging");
        if (rc) return rc;
    }
    int rc = copy_in(rho_r, on_device, N * es, &d_rr, scratch, h->stream);
    if (!rc) rc = copy_in(rho_b, on_device, N * es, &d_rb, scratch ? (char*)scratch + N * es : nullptr, h->stream);
    if (!rc && u) rc = copy_in(u, on_device, 3 * N * es, &d_u, scratch ? (char*)scratch + 2 * N * es : nullptr, h->stream);
    if (!rc) {
        LatticeView v = view_of(h);
        rc = launch_init(v, d_rr, d_rb, d_u, dtype);
    }
    if (scratch) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(scratch);
    }
    if (rc) return rc;
    h->initialised = true;
    h->fresh = true;
    h->part_valid = false;
    h->steps = 0;
    return LB_OK;
}

int lb_init_droplets(lb_t* h, const double* centres, const double* radii, int32_t n, double width,
                     double background, double rho0) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (n < 0 || (n > 0 && (!centres || !radii))) return fail(LB_EINVAL, "bad droplet list");
    if (!(width > 0.0) || !(rho0 > 0.0) || !(background >= -1.0 && background <= 1.0))
        return fail(LB_EINVAL, "width and rho0 must be > 0, background in [-1, 1]");
    for (int32_t j = 0; j < n; ++j)
        if (!(radii[j] >= 0.0) || !std::isfinite(centres[3 * j] + centres[3 * j + 1] + centres[3 * j + 2]))
            return fail(LB_EINVAL, "droplet radii must be >= 0 and centres finite");
    const size_t N = (size_t)h->g.N;
    const bool split = h->p.storage >= LB_STORE_F16;
    if (split && !h->pending) {
        int rc = check_hip(hipMalloc(&h->pending, pop_bytes(LB_STORE_F32, N)), "hipMalloc initial state");
        if (rc) return rc;
    }
    double* tmp = nullptr;
    const size_t bytes = (2 * N + 4 * (size_t)n + 4) * sizeof(double);
    int rc = check_hip(hipMalloc((void**)&tmp, bytes), "hipMalloc droplet staging");
    if (rc) return rc;
    double* rr = tmp;
    double* rb = tmp + N;
    double* dc = tmp + 2 * N;
    double* dr = dc + 3 * (size_t)n;
    if (n) rc = check_hip(hipMemcpyAsync(dc, centres, 3 * sizeof(double) * n, hipMemcpyHostToDevice, h->stream), "H2D");
    if (!rc && n) rc = check_hip(hipMemcpyAsync(dr, radii, sizeof(double) * n, hipMemcpyHostToDevice, h->stream), "H2D");
    if (!rc) rc = launch_droplets(h->stream, h->g, dc, dr, n, width, background, rho0, rr, rb);
    if (!rc) {
        LatticeView v = view_of(h);
        rc = launch_init(v, rr, rb, nullptr, LB_DTYPE_F64);
    }
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(tmp);
    if (rc) return rc;
    h->initialised = true;
    h->fresh = true;
    h->part_valid = false;
    h->steps = 0;
    return LB_OK;
}

// One step of lattice h (events t may be null); `used` receives the kernel
// that ran.
static int advance(lb_t* h, const StepEvents* t, int* used) {
    LatticeView v = view_of(h);
    // the first step of a 16-bit lattice with moving walls (from its raw
    // initial state) takes two passes: the one-read kernel of that step does
    // not gather the wall terms the next step's pull adds
    const bool first16 = h->g.moving && h->pending;
    const int kernel = (h->kernel == LB_KERNEL_FUSED && first16) ? LB_KERNEL_TWOPASS : h->kernel;
    int rc = launch_step(v, kernel, t);
    if (rc) return rc;
    if (h->pending) {
        // the first step consumed the raw initial state
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(h->pending);
        h->pending = nullptr;
    }
    h->cur ^= 1;
    h->steps++;
    h->fresh = false;
    if (kernel == LB_KERNEL_FUSED) {
        const FusedShape fs = tile_shape(h->p, TILE_SINGLE);
        h->part_cur ^= 1;
        h->part_valid = true;
        h->part_ty = fs.TY;
        h->part_tz = fs.TZ;
    } else {
        h->part_valid = false;
    }
    if (used) *used = kernel;
    return LB_OK;
}

int lb_step(lb_t* h, int32_t n) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (n < 0) return fail(LB_EINVAL, "n must be >= 0");
    if (!h->initialised) return fail(LB_ESTATE, "lb_step before lb_init_fields");
    for (int32_t k = 0; k < n; ++k) {
        int rc = advance(h, nullptr, nullptr);
        if (rc) return rc;
    }
    return LB_OK;
}

int lb_step_timed(lb_t* h, int32_t n, double kernel_ms[3]) {
    if (!h || !kernel_ms) return fail(LB_EINVAL, "NULL argument");
    if (n < 1) return fail(LB_EINVAL, "n must be >= 1");
    if (!h->initialised) return fail(LB_ESTATE, "lb_step_timed before lb_init_fields");
    StepEvents* ev = new (std::nothrow) StepEvents[n]();
    if (!ev) return fail(LB_ENOMEM, "host allocation failed");
    int rc = LB_OK;
    int made = 0;
    for (; made < n && !rc; ++made)
        for (int k = 0; k < 3 && !rc; ++k) rc = check_hip(hipEventCreate(&ev[made].ev[k]), "hipEventCreate");
    int* used = new (std::nothrow) int[n]();
    if (!used) rc = fail(LB_ENOMEM, "host allocation failed");
    for (int32_t k = 0; k < n && !rc; ++k) rc = advance(h, &ev[k], &used[k]);
    if (!rc) rc = check_hip(hipStreamSynchronize(h->stream), "sync");
    double a = 0, b = 0, c = 0;
    if (!rc) {
        for (int32_t k = 0; k < n; ++k) {
            // two-pass: [0] phase pass, [1] collide pass; one-read: [0] the phase
            // assembly (and the own sums of a state no one-read step made), [1]
            // the collide tile
            float t01 = 0, t12 = 0, t02 = 0;
            (void)hipEventElapsedTime(&t01, ev[k].ev[0], ev[k].ev[1]);
            (void)hipEventElapsedTime(&t12, ev[k].ev[1], ev[k].ev[2]);
            (void)hipEventElapsedTime(&t02, ev[k].ev[0], ev[k].ev[2]);
            a += t01;
            b += t12;
            c += t02;
        }
        kernel_ms[0] = a / n;
        kernel_ms[1] = b / n;
        kernel_ms[2] = c / n;
    }
    for (int k = 0; k < n; ++k)
        for (int e = 0; e < 3; ++e)
            if (ev[k].ev[e]) (void)hipEventDestroy(ev[k].ev[e]);
    delete[] ev;
    delete[] used;
    return rc;
}

int lb_moments(lb_t* h, void* rho_r, void* rho_b, void* mom, int32_t dtype, int32_t on_device,
               double totals[14]) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (!h->initialised) return fail(LB_ESTATE, "lb_moments before lb_init_fields");
    if (dtype != LB_DTYPE_F64 && dtype != LB_DTYPE_F32) return fail(LB_EINVAL, "bad dtype");
    const size_t N = (size_t)h->g.N;
    const size_t es = dtype == LB_DTYPE_F64 ? 8 : 4;
    LatticeView v = view_of(h);
    int rc = LB_OK;
    if (rho_r || rho_b || mom) {
        void* scratch = nullptr;
        if (!on_device) {
            rc = check_hip(hipMalloc(&scratch, 5 * N * es), "hipMalloc staging");
            if (rc) return rc;
        }
        char* base = (char*)scratch;
        void* o_rr = rho_r ? (on_device ? rho_r : base) : nullptr;
        void* o_rb = rho_b ? (on_device ? rho_b : base + N * es) : nullptr;
        void* o_j = mom ? (on_device ? mom : base + 2 * N * es) : nullptr;
        rc = launch_moments(v, o_rr, o_rb, o_j, dtype);
        if (!rc && !on_device) {
            if (rho_r) rc = check_hip(hipMemcpyAsync(rho_r, o_rr, N * es, hipMemcpyDeviceToHost, h->stream), "D2H");
            if (!rc && rho_b) rc = check_hip(hipMemcpyAsync(rho_b, o_rb, N * es, hipMemcpyDeviceToHost, h->stream), "D2H");
            if (!rc && mom) rc = check_hip(hipMemcpyAsync(mom, o_j, 3 * N * es, hipMemcpyDeviceToHost, h->stream), "D2H");
            if (!rc) rc = check_hip(hipStreamSynchronize(h->stream), "sync");
        }
        if (scratch) {
            (void)hipStreamSynchronize(h->stream);
            (void)hipFree(scratch);
        }
        if (rc) return rc;
    }
    if (totals) {
        rc = launch_totals(v, h->partial, h->dtot);
        if (!rc) rc = check_hip(hipMemcpyAsync(totals, h->dtot, sizeof(double) * 2 * NTOT, hipMemcpyDeviceToHost, h->stream), "D2H totals");
        if (!rc) rc = check_hip(hipStreamSynchronize(h->stream), "sync");
    }
    return rc;
}

int lb_korteweg(lb_t* h, double lambda, int32_t b, void* k_blocks, void* phi_blocks, int32_t dtype,
                int32_t on_device, int32_t accumulate) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (!h->initialised) return fail(LB_ESTATE, "lb_korteweg before lb_init_fields");
    if (dtype != LB_DTYPE_F64 && dtype != LB_DTYPE_F32) return fail(LB_EINVAL, "bad dtype");
    if (!k_blocks && !phi_blocks) return fail(LB_EINVAL, "no output");
    if (b != 1 && b != 2 && b != 4 && b != 8) return fail(LB_EINVAL, "block size must be 1, 2, 4 or 8");
    if (h->p.nx % b || h->p.ny % b || h->p.nz % b) return fail(LB_EINVAL, "lattice extents are not multiples of b");
    if (accumulate && !on_device) return fail(LB_EINVAL, "accumulation needs device outputs");
    if (!std::isfinite(lambda)) return fail(LB_EINVAL, "lambda must be finite");
    const size_t Nc = (size_t)(h->p.nx / b) * (h->p.ny / b) * (h->p.nz / b);
    const size_t es = dtype == LB_DTYPE_F64 ? 8 : 4;
    LatticeView v = view_of(h);
    void* scratch = nullptr;
    if (!on_device) {
        int rc = check_hip(hipMalloc(&scratch, 7 * Nc * es), "hipMalloc staging");
        if (rc) return rc;
    }
    void* ko = k_blocks ? (on_device ? k_blocks : scratch) : nullptr;
    void* po = phi_blocks ? (on_device ? phi_blocks : (char*)scratch + 6 * Nc * es) : nullptr;
    int rc = launch_korteweg(v, lambda, b, ko, po, dtype, accumulate);
    if (!rc && !on_device) {
        if (k_blocks) rc = check_hip(hipMemcpyAsync(k_blocks, ko, 6 * Nc * es, hipMemcpyDeviceToHost, h->stream), "D2H");
        if (!rc && phi_blocks)
            rc = check_hip(hipMemcpyAsync(phi_blocks, po, Nc * es, hipMemcpyDeviceToHost, h->stream), "D2H");
        if (!rc) rc = check_hip(hipStreamSynchronize(h->stream), "sync");
    }
    if (scratch) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(scratch);
    }
    return rc;
}

int lb_get_state(lb_t* h, void* f, int32_t dtype, int32_t on_device) {
    if (!h || !f) return fail(LB_EINVAL, "NULL argument");
    if (!h->initialised) return fail(LB_ESTATE, "lb_get_state before lb_init_fields");
    if (dtype != LB_DTYPE_F64 && dtype != LB_DTYPE_F32) return fail(LB_EINVAL, "bad dtype");
    const size_t bytes = 2 * Q * (size_t)h->g.N * (dtype == LB_DTYPE_F64 ? 8 : 4);
    void* out = f;
    if (!on_device) {
        int rc = check_hip(hipMalloc(&out, bytes), "hipMalloc staging");
        if (rc) return rc;
    }
    LatticeView v = view_of(h);
    int rc = launch_export(v, out, dtype);
    if (!rc && !on_device) {
        rc = check_hip(hipMemcpyAsync(f, out, bytes, hipMemcpyDeviceToHost, h->stream), "D2H state");
        if (!rc) rc = check_hip(hipStreamSynchronize(h->stream), "sync");
    }
    if (!on_device) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(out);
    }
    return rc;
}

int lb_set_state(lb_t* h, const void* f, int32_t dtype, int32_t on_device) {
    if (!h || !f) return fail(LB_EINVAL, "NULL argument");
    if (dtype != LB_DTYPE_F64 && dtype != LB_DTYPE_F32) return fail(LB_EINVAL, "bad dtype");
    const size_t N = (size_t)h->g.N;
    const size_t bytes = 2 * Q * N * (dtype == LB_DTYPE_F64 ? 8 : 4);
    const bool split = h->p.storage >= LB_STORE_F16;
    if (split && !h->pending) {
        int rc = check_hip(hipMalloc(&h->pending, pop_bytes(LB_STORE_F32, N)), "hipMalloc raw state");
        if (rc) return rc;
    }
    const void* in = f;
    void* staging = nullptr;
    if (!on_device) {
        int rc = check_hip(hipMalloc(&staging, bytes), "hipMalloc staging");
        if (!rc) rc = check_hip(hipMemcpyAsync(staging, f, bytes, hipMemcpyHostToDevice, h->stream), "H2D state");
        if (rc) {
            if (staging) (void)hipFree(staging);
            return rc;
        }
        in = staging;
    }
    LatticeView v = view_of(h);
    int rc = launch_import(v, in, dtype);
    if (staging) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(staging);
    }
    if (rc) return rc;
    h->initialised = true;
    h->fresh = true;
    h->part_valid = false;
    return LB_OK;
}

int64_t lb_state_bytes(const lb_t* h) {
    if (!h) return -1;
    return (int64_t)pop_bytes(h->p.storage, (size_t)h->g.N);
}

int lb_save_raw(lb_t* h, void* dst, int32_t on_device) {
    if (!h || !dst) return fail(LB_EINVAL, "NULL argument");
    if (!h->initialised) return fail(LB_ESTATE, "no state yet");
    if (h->pending) return fail(LB_ESTATE, "16-bit lattice holds a raw initial state until its first step; use lb_get_state");
    const size_t b = pop_bytes(h->p.storage, (size_t)h->g.N);
    int rc = check_hip(hipMemcpyAsync(dst, h->buf[h->cur], b, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream), "copy raw state");
    if (!rc && !on_device) rc = check_hip(hipStreamSynchronize(h->stream), "sync");
    return rc;
}

int lb_load_raw(lb_t* h, const void* src, int32_t on_device) {
    if (!h || !src) return fail(LB_EINVAL, "NULL argument");
    const size_t b = pop_bytes(h->p.storage, (size_t)h->g.N);
    int rc = check_hip(hipMemcpyAsync(h->buf[h->cur], src, b, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->stream), "copy raw state");
    if (!rc && !on_device) rc = check_hip(hipStreamSynchronize(h->stream), "sync");
    if (rc) return rc;
    if (h->pending) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(h->pending);
        h->pending = nullptr;
    }
    h->initialised = true;
    h->fresh = false;
    h->part_valid = false;
    return LB_OK;
}

int64_t lb_step_count(const lb_t* h) { return h ? h->steps : -1; }

int lb_kernel_in_use(const lb_t* h) { return h ? h->kernel : LB_EINVAL; }

}  // extern "C"
