// lb_internal.hpp -- declarations shared by the host translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "lb.h"
#include "lb_single.hpp"

namespace lbm {

// Blocks of the compensated-reduction kernel (fixed, so totals are bitwise
// reproducible for a given lattice).
constexpr int kTotalsBlocks = 512;

// What a launch needs to know about one lattice.
struct LatticeView {
    const lb_params* p = nullptr;
    Geom g;
    hipStream_t stream = nullptr;
    void* cur = nullptr;       // post-collision buffer holding the current state
    void* nxt = nullptr;       // buffer the next step writes
    void* pending = nullptr;   // raw FP32 current state of a 16-bit lattice (else null)
    void* phi = nullptr;       // phase-field scratch of the two-pass step
    void* part_in = nullptr;   // phase sums and phase field of the current state (one-read step)
    void* part_out = nullptr;  // the same, written by the one-read step for the next state
    bool part_valid = false;   // part_in holds the current state's sums
    bool shape_set = false;    // the one-read step uses `shape` (not the lattice's own tile shape)
    FusedShape shape{};
    Coeffs<double> cd;
    Coeffs<float> cf;
};

int set_error(int code, const char* msg);
int validate_params(const lb_params* p, std::string& why);
template <typename R>
Coeffs<R> make_coeffs(const lb_params& p);
Geom make_geom(const lb_params& p);
size_t pop_bytes(int storage, size_t N);

// Tile kernels: 64-wide tiles of TY rows marching z-chunks of TZ planes.
constexpr int kTX = 64;
enum TileKind { TILE_COLLIDE = 0, TILE_SINGLE = 1, TILE_PHASE = 2, TILE_BATCH = 3 };
// Tile shape set through lb_set_tiles for (kind, storage): 0 = unset.
struct TileSetting {
    int ty, tz;
};
TileSetting tile_setting(int kind, int storage);
void set_tile_setting(int kind, int storage, int ty, int tz);
int env_int(const char* name, int dflt);
int tile_halo(const lb_params& p);
size_t tile_lds(const lb_params& p, int kind, int TY);
int tile_rows(const lb_params& p, int kind);
FusedShape tile_shape(const lb_params& p, int kind, int target_blocks = 1024);

int choose_kernel(const lb_params& p);
// Events recorded around the passes of one step (null = no timing):
// ev[0] before the step, ev[1] between the phase and the collide pass (equal
// to ev[0] for the fused kernel), ev[2] after the step.
struct StepEvents {
    hipEvent_t ev[3];
};
int launch_step(const LatticeView& v, int kernel, const StepEvents* t = nullptr);
// Tile kernel of the one-read step for raw storage (lb_lean.hip): collide and
// stream fin into fout, gathering the next state's own phase sums.
template <typename T>
int launch_lean(const LatticeView& v, const T* fin, T* fout, const Coeffs<T>& c, const FusedShape& fs);
// The same for 16-bit moment-split storage (lb_lean16.hip).
template <typename H>
int launch_lean_split(const LatticeView& v, const SplitPop<H>& src, const SplitPop<H>& dst, const Coeffs<float>& c,
                      const FusedShape& fs);
int launch_init(const LatticeView& v, const void* rr, const void* rb, const void* u, int dtype);
int launch_import(const LatticeView& v, const void* f, int dtype);
int launch_export(const LatticeView& v, void* out, int dtype);
int launch_moments(const LatticeView& v, void* rr, void* rb, void* j, int dtype);
int launch_korteweg(const LatticeView& v, double lam, int b, void* kout, void* pout, int dtype, int accumulate);
int launch_totals(const LatticeView& v, Neu* partial, double* dtot);
int launch_droplets(hipStream_t st, const Geom& g, const double* cen, const double* rad, int n, double width,
                    double background, double rho0, double* rr, double* rb);

}  // namespace lbm
