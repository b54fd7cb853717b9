// lb_batch.hip -- many independent lattices (jobs) advanced together: each
// step is one persistent assembly launch and two persistent tile launches
// (jobs without walls, jobs with walls), each walking a work list of
// (job, item) pairs with the same code as the one-read step of a single
// lattice (assemble_site, lean_tile), then a one-thread tick; steps are
// replayed from a captured HIP graph.
//
// Each job has a window [first, last) of global steps.  A device counter holds
// the global step; the step kernels read it, skip jobs outside their window
// and pick each job's ping-pong buffers (populations and phase sums) from
// (step - first) parity, and the tick advances it.  The graph therefore never
// changes: admitting or removing a job only rewrites the job table and the
// work lists (ordered on the batch stream), so jobs join and leave between
// replays.  Admission takes a job's first step on its own, through the single
// lattice's one-read step with the batch's tile boxes, so that the job enters
// the batch with the phase sums of its current state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "lb.h"
#include "lb_internal.hpp"
#include "lb_lean.hpp"

using namespace lbm;

namespace lbm {

constexpr int kBatchH = 3;   // halo for near-contact ranges up to 2
constexpr int kAsmThreads = 256;

template <typename R>
struct BatchJob {
    Geom g;
    Coeffs<R> c;
    FusedShape fs;
    FaceSet faces;          // face sites of the job's tile boxes (assembly)
    void* buf[2];           // populations, ping-pong
    void* part[2];          // phase sums and phase field of the state in buf[k]
    long long first, last;  // global-step window
    int active;
    int tiles;              // tiles_x * tiles_y
    float scale;            // 16-bit deviation scale 2^scale_log2 of this job (1 otherwise)
};

// A tile item: block = tile + tiles * chunk.  An assembly item: block = index
// of a run of kAsmThreads face sites.
struct WorkItem {
    int slot;
    int block;
};

// Storage views of a job's buffers: the assembly's source view, and the
// lean tile's policy from the source and destination buffers.
template <typename H>
__device__ __forceinline__ SplitPop<H> split_storage_view(void* buf, size_t N, float scale) {
    SplitPop<H> s;
    s.rec = (float*)buf;
    s.dev = (H*)((float*)buf + 8 * N);
    s.N = N;
    s.scale = scale;
    s.inv_scale = 1.0f / scale;
    return s;
}

template <typename S>
struct BatchStorage;
template <typename T>
struct BatchStorage<LeanRaw<T>> {
    using Src = RawPop<T>;
    static __device__ __forceinline__ Src view(void* buf, size_t N, float) { return Src{(T*)buf, N}; }
    static __device__ __forceinline__ LeanRaw<T> policy(void* in, void* out, size_t, float, f4*, int) {
        return LeanRaw<T>{(const T*)in, (T*)out};
    }
};
template <typename H>
struct BatchStorage<LeanSplit<H>> {
    using Src = SplitPop<H>;
    static __device__ __forceinline__ Src view(void* buf, size_t N, float scale) {
        return split_storage_view<H>(buf, N, scale);
    }
    static __device__ __forceinline__ LeanSplit<H> policy(void* in, void* out, size_t N, float scale, f4* ring,
                                                          int TY) {
        const SplitPop<H> a = split_storage_view<H>(in, N, scale), b = split_storage_view<H>(out, N, scale);
        LeanSplit<H> st;
        st.rin = a.rec;
        st.din = a.dev;
        st.rout = b.rec;
        st.dout = b.dev;
        st.codec = a;
        st.ring = ring;
        st.TY = TY;
        return st;
    }
};

// Workgroup b of a persistent launch takes items b', b' + G, ... where b'
// spreads contiguous item runs over the 8 XCDs so neighbouring tiles of a job
// share an L2.
__device__ __forceinline__ int persistent_start() {
    const int G = gridDim.x;
    int b = blockIdx.x;
    if ((G & 7) == 0) b = (b & 7) * (G >> 3) + (b >> 3);
    return b;
}

template <typename R>
__device__ __forceinline__ bool job_live(const BatchJob<R>& J, long long gs) {
    return J.active && gs >= J.first && gs < J.last;
}

// Assembly: phi of the face sites of every live job's current state.  The
// work list holds n_items[0] tile items of jobs without walls, then
// n_items[1] tile items of jobs with walls, then n_items[2] assembly items.
template <typename R, typename S, int TY>
__global__ __launch_bounds__(kAsmThreads) void batch_assemble_kernel(const BatchJob<R>* __restrict__ jobs,
                                                                     const WorkItem* __restrict__ items,
                                                                     const int* __restrict__ n_items,
                                                                     const long long* __restrict__ gstep) {
    using B = BatchStorage<S>;
    const int n0 = n_items[0] + n_items[1], n = n_items[2];
    const long long gs = *gstep;
    for (int w = persistent_start(); w < n; w += gridDim.x) {
        const WorkItem it = items[n0 + w];
        const BatchJob<R>& J = jobs[it.slot];
        if (!job_live(J, gs)) continue;  // uniform over the workgroup
        const int par = (int)((gs - J.first) & 1);
        const typename B::Src src = B::view(J.buf[par], (size_t)J.g.N, J.scale);
        assemble_site<R, typename B::Src, kTX, TY>(J.g, src, J.faces, (Part2<R>*)J.part[par],
                                                  it.block * kAsmThreads + (int)threadIdx.x);
    }
}

// LDS of the batch tile kernel: that of a lean tile with the batch halo.
template <typename S, int TY>
__host__ __device__ constexpr size_t batch_lds_bytes() {
    return lean_lds_bytes<S, TY, kBatchH>();
}

// Tiles: collide, stream and gather the next state's phase sums of every
// live job's tile items, jobs with walls (W) or without them (the two tile
// variants in one kernel would hold the registers of both).
template <typename S, int TY, bool W>
__global__ __launch_bounds__(kTX * TY) void batch_tile_kernel(const BatchJob<typename S::R>* __restrict__ jobs,
                                                              const WorkItem* __restrict__ items,
                                                              const int* __restrict__ n_items,
                                                              const long long* __restrict__ gstep) {
    using R = typename S::R;
    using B = BatchStorage<S>;
    extern __shared__ unsigned char lds_raw[];
    R* ringb = reinterpret_cast<R*>(lds_raw);
    size_t off = (phi_ring_bytes<R, kTX, kBatchH>(TY) + 15) & ~size_t(15);
    f4* rec_ring = reinterpret_cast<f4*>(lds_raw + off);
    off += S::ring_bytes(TY);
    R* xch = reinterpret_cast<R*>(lds_raw + off);
    Part2<R>* vs = reinterpret_cast<Part2<R>*>(lds_raw + off + lean_xch_bytes<R, TY>());
    const int first = W ? n_items[0] : 0, n = n_items[W ? 1 : 0];
    const long long gs = *gstep;
    for (int w = persistent_start(); w < n; w += gridDim.x) {
        const WorkItem it = items[first + w];
        const BatchJob<R>& J = jobs[it.slot];
        if (!job_live(J, gs)) continue;  // uniform over the workgroup
        const int par = (int)((gs - J.first) & 1);
        const Geom g = J.g;
        const S st = B::policy(J.buf[par], J.buf[par ^ 1], (size_t)g.N, J.scale, rec_ring, TY);
        const int tile = it.block % J.tiles, chunk = it.block / J.tiles;
        const int x0 = (tile % J.fs.tiles_x) * kTX, y0 = (tile / J.fs.tiles_x) * TY;
        const int za = chunk * J.fs.TZ, zb = min(za + J.fs.TZ, g.nz);
        Part2<R>* const pin = (Part2<R>*)J.part[par];
        Part2<R>* const pout = (Part2<R>*)J.part[par ^ 1];
        lean_tile<S, TY, kBatchH, W>(g, st, J.c, ringb, xch, vs, x0, y0, za, zb, phi_of<kTX>(pin, g), pout,
                                     phi_of<kTX>(pout, g), 0);  // (batched jobs have no moving walls)
        __syncthreads();  // the next item restages every LDS ring
    }
}

__global__ void batch_tick_kernel(long long* gstep) {
    if (blockIdx.x == 0 && threadIdx.x == 0) gstep[0] = gstep[0] + 1;
}

// Tile rows of the batched step: 8 (4 on request); the lean tile is
// instantiated for these two.
int batch_rows(int want) { return want > 0 && want < 8 ? 4 : 8; }

size_t batch_tile_lds(int storage, int TY) {
    switch (storage) {
        case LB_STORE_F64: return TY == 4 ? batch_lds_bytes<LeanRaw<double>, 4>() : batch_lds_bytes<LeanRaw<double>, 8>();
        case LB_STORE_F32: return TY == 4 ? batch_lds_bytes<LeanRaw<float>, 4>() : batch_lds_bytes<LeanRaw<float>, 8>();
        default:
            return TY == 4 ? batch_lds_bytes<LeanSplit<__half>, 4>() : batch_lds_bytes<LeanSplit<__half>, 8>();
    }
}

}  // namespace lbm

namespace {

thread_local std::string g_berr;

int bfail(int code, const std::string& m) {
    lbm::set_error(code, m.c_str());
    return code;
}

int bcheck(hipError_t e, const char* what) {
    if (e == hipSuccess) return LB_OK;
    return bfail(e == hipErrorOutOfMemory ? LB_ENOMEM : LB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// First-fit allocator over the arena, 256-byte granules, coalescing on free.
struct Arena {
    size_t size = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    void reset(size_t n) {
        size = n;
        free_.clear();
        if (n) free_[0] = n;
    }
    bool alloc(size_t n, size_t& off) {
        n = (n + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                off = it->first;
                const size_t rest = it->second - n;
                free_.erase(it);
                if (rest) free_[off + n] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = (n + 255) & ~size_t(255);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const {
        size_t m = 0;
        for (auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }
};

struct HostJob {
    bool used = false;
    lb_params p;
    size_t off = 0, bytes = 0;
    long long first = 0, last = 0;
    Coeffs<double> cd;
    Coeffs<float> cf;
    FusedShape fs;
};

}  // namespace

struct lb_batch_t {
    int max_jobs;
    int storage;
    int graph_steps;
    hipStream_t stream;
    char* arena_base = nullptr;
    Arena arena;
    std::vector<HostJob> jobs;
    void* d_jobs = nullptr;     // BatchJob<R>[max_jobs]
    WorkItem* d_items = nullptr;  // tile items, then assembly items
    int* d_nitems = nullptr;      // [3]: tile items without walls, with walls, assembly items
    long long* d_gstep = nullptr;
    int items_cap = 0;
    long long gstep = 0;        // host mirror of the device counter
    void* staging = nullptr;    // raw FP32 initial state / host field staging
    size_t staging_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int grid = 0;               // workgroups of the persistent tile launch (all resident)
    int agrid = 0;              // workgroups of the persistent assembly launch
    int ty = 8, tz = 32;        // tile rows and chunk planes of every job (fixed at creation)
    bool own_stream = false;
};

namespace {

// Two population buffers and two phase-sum buffers.
size_t job_half(int storage, size_t N) { return (lbm::pop_bytes(storage, N) + 255) & ~size_t(255); }

size_t job_part(const lb_params& p) {
    return (part_reals<kTX>(p.nx, p.ny, p.nz) * (p.storage == LB_STORE_F64 ? 8 : 4) + 255) & ~size_t(255);
}

size_t job_bytes(const lb_params& p) {
    return 2 * job_half(p.storage, (size_t)p.nx * p.ny * p.nz) + 2 * job_part(p);
}

float batch_scale(const lb_batch_t* b, const lb_params& p) {
    return b->storage == LB_STORE_F16 ? std::ldexp(1.0f, p.scale_log2 ? p.scale_log2 : 16) : 1.0f;
}

FusedShape job_shape(const lb_batch_t* b, const lb_params& p) {
    FusedShape fs;
    fs.TY = b->ty;
    fs.tiles_x = (p.nx + kTX - 1) / kTX;
    fs.tiles_y = (p.ny + fs.TY - 1) / fs.TY;
    fs.TZ = std::min(p.nz, b->tz);
    fs.chunks = (p.nz + fs.TZ - 1) / fs.TZ;
    fs.nblocks = fs.tiles_x * fs.tiles_y * fs.chunks;
    return fs;
}

template <typename R>
void fill_desc(const lb_batch_t* b, const HostJob& h, BatchJob<R>& d) {
    std::memset(&d, 0, sizeof(d));
    d.g = make_geom(h.p);
    if constexpr (std::is_same<R, double>::value)
        d.c = h.cd;
    else
        d.c = h.cf;
    d.fs = h.fs;
    d.faces = face_set(d.g, kTX, h.fs.TY, h.fs.TZ);
    const size_t half = job_half(b->storage, (size_t)h.p.nx * h.p.ny * h.p.nz), part = job_part(h.p);
    char* base = b->arena_base + h.off;
    d.buf[0] = base;
    d.buf[1] = base + half;
    d.part[0] = base + 2 * half;
    d.part[1] = base + 2 * half + part;
    d.first = h.first;
    d.last = h.last;
    d.active = h.used ? 1 : 0;
    d.tiles = h.fs.tiles_x * h.fs.tiles_y;
    d.scale = batch_scale(b, h.p);
}

size_t desc_size(int storage) { return storage == LB_STORE_F64 ? sizeof(BatchJob<double>) : sizeof(BatchJob<float>); }

int upload_desc(lb_batch_t* b, int slot) {
    alignas(16) unsigned char tmp[sizeof(BatchJob<double>)];
    if (b->storage == LB_STORE_F64)
        fill_desc<double>(b, b->jobs[slot], *reinterpret_cast<BatchJob<double>*>(tmp));
    else
        fill_desc<float>(b, b->jobs[slot], *reinterpret_cast<BatchJob<float>*>(tmp));
    const size_t ds = desc_size(b->storage);
    int rc = bcheck(hipMemcpyAsync((char*)b->d_jobs + ds * slot, tmp, ds, hipMemcpyHostToDevice, b->stream), "upload job");
    if (!rc) rc = bcheck(hipStreamSynchronize(b->stream), "sync");
    return rc;
}

bool has_walls(const lb_params& p) { return p.bc[0] || p.bc[1] || p.bc[2]; }

int upload_items(lb_batch_t* b) {
    std::vector<WorkItem> items;
    int counts[3] = {0, 0, 0};
    for (int pass = 0; pass < 2; ++pass) {
        // tile items of the jobs without walls, then of those with walls
        for (int s = 0; s < b->max_jobs; ++s) {
            const HostJob& h = b->jobs[s];
            if (!h.used || has_walls(h.p) != (pass == 1)) continue;
            for (int k = 0; k < h.fs.nblocks; ++k) items.push_back(WorkItem{s, k});
        }
        counts[pass] = (int)items.size() - (pass ? counts[0] : 0);
    }
    for (int s = 0; s < b->max_jobs; ++s) {
        const HostJob& h = b->jobs[s];
        if (!h.used) continue;
        const FaceSet f = face_set(make_geom(h.p), kTX, h.fs.TY, h.fs.TZ);
        const int runs = (f.row_sites + f.edge_sites + kAsmThreads - 1) / kAsmThreads;
        for (int k = 0; k < runs; ++k) items.push_back(WorkItem{s, k});
    }
    counts[2] = (int)items.size() - counts[0] - counts[1];
    if ((int)items.size() > b->items_cap) {
        // grow the work list; the graph holds its pointer, so drop the graph
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        int rc = bcheck(hipStreamSynchronize(b->stream), "sync");
        if (rc) return rc;
        if (b->d_items) (void)hipFree(b->d_items);
        b->d_items = nullptr;
        int cap = std::max<int>(1024, (int)items.size() * 2);
        rc = bcheck(hipMalloc((void**)&b->d_items, sizeof(WorkItem) * cap), "hipMalloc work list");
        if (rc) return rc;
        b->items_cap = cap;
    }
    int n = (int)items.size();
    int rc = LB_OK;
    if (n) rc = bcheck(hipMemcpyAsync(b->d_items, items.data(), sizeof(WorkItem) * n, hipMemcpyHostToDevice, b->stream), "upload work list");
    if (!rc) rc = bcheck(hipMemcpyAsync(b->d_nitems, counts, sizeof(counts), hipMemcpyHostToDevice, b->stream), "upload counts");
    if (!rc) rc = bcheck(hipStreamSynchronize(b->stream), "sync");
    return rc;
}

template <typename S, int TY, bool W>
const void* tile_kernel_of() {
    return reinterpret_cast<const void*>(batch_tile_kernel<S, TY, W>);
}

template <typename S, int TY>
int launch_batch_ty(lb_batch_t* b) {
    using R = typename S::R;
    hipLaunchKernelGGL((batch_assemble_kernel<R, S, TY>), dim3(b->agrid), dim3(kAsmThreads), 0, b->stream,
                       (const BatchJob<R>*)b->d_jobs, b->d_items, b->d_nitems, b->d_gstep);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(LB_EDEVICE, std::string("batch_assemble_kernel: ") + hipGetErrorString(e));
    const size_t lds = batch_lds_bytes<S, TY>();
    hipLaunchKernelGGL((batch_tile_kernel<S, TY, false>), dim3(b->grid), dim3(kTX * TY), lds, b->stream,
                       (const BatchJob<R>*)b->d_jobs, b->d_items, b->d_nitems, b->d_gstep);
    e = hipGetLastError();
    if (e != hipSuccess) return bfail(LB_EDEVICE, std::string("batch_tile_kernel: ") + hipGetErrorString(e));
    hipLaunchKernelGGL((batch_tile_kernel<S, TY, true>), dim3(b->grid), dim3(kTX * TY), lds, b->stream,
                       (const BatchJob<R>*)b->d_jobs, b->d_items, b->d_nitems, b->d_gstep);
    e = hipGetLastError();
    if (e != hipSuccess) return bfail(LB_EDEVICE, std::string("batch_tile_kernel: ") + hipGetErrorString(e));
    hipLaunchKernelGGL(batch_tick_kernel, dim3(1), dim3(64), 0, b->stream, b->d_gstep);
    e = hipGetLastError();
    if (e != hipSuccess) return bfail(LB_EDEVICE, std::string("batch_tick_kernel: ") + hipGetErrorString(e));
    return LB_OK;
}

template <typename S>
int launch_batch_step(lb_batch_t* b) {
    return b->ty == 4 ? launch_batch_ty<S, 4>(b) : launch_batch_ty<S, 8>(b);
}

int batch_step_once(lb_batch_t* b) {
    switch (b->storage) {
        case LB_STORE_F64: return launch_batch_step<LeanRaw<double>>(b);
        case LB_STORE_F32: return launch_batch_step<LeanRaw<float>>(b);
        case LB_STORE_F16: return launch_batch_step<LeanSplit<__half>>(b);
        case LB_STORE_BF16: return launch_batch_step<LeanSplit<__hip_bfloat16>>(b);
    }
    return bfail(LB_EINVAL, "unknown storage");
}

// A tile kernel of the batch (for its LDS opt-in and occupancy).
template <bool W>
const void* batch_tile_kernel_of(int storage, int TY) {
    switch (storage) {
        case LB_STORE_F64:
            return TY == 4 ? tile_kernel_of<LeanRaw<double>, 4, W>() : tile_kernel_of<LeanRaw<double>, 8, W>();
        case LB_STORE_F32:
            return TY == 4 ? tile_kernel_of<LeanRaw<float>, 4, W>() : tile_kernel_of<LeanRaw<float>, 8, W>();
        case LB_STORE_F16:
            return TY == 4 ? tile_kernel_of<LeanSplit<__half>, 4, W>() : tile_kernel_of<LeanSplit<__half>, 8, W>();
        default:
            return TY == 4 ? tile_kernel_of<LeanSplit<__hip_bfloat16>, 4, W>()
                           : tile_kernel_of<LeanSplit<__hip_bfloat16>, 8, W>();
    }
}

int ensure_graph(lb_batch_t* b) {
    if (b->exec) return LB_OK;
    int rc = bcheck(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (rc) return rc;
    for (int k = 0; k < b->graph_steps && !rc; ++k) rc = batch_step_once(b);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return bcheck(e, "hipStreamEndCapture");
    rc = bcheck(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "hipGraphInstantiate");
    if (rc) {
        (void)hipGraphDestroy(g);
        return rc;
    }
    b->graph = g;
    return LB_OK;
}

int ensure_staging(lb_batch_t* b, size_t bytes) {
    if (b->staging_bytes >= bytes) return LB_OK;
    int rc = bcheck(hipStreamSynchronize(b->stream), "sync");
    if (rc) return rc;
    if (b->staging) (void)hipFree(b->staging);
    b->staging = nullptr;
    b->staging_bytes = 0;
    rc = bcheck(hipMalloc(&b->staging, bytes), "hipMalloc staging");
    if (!rc) b->staging_bytes = bytes;
    return rc;
}

LatticeView job_view(lb_batch_t* b, int slot, void* cur, void* nxt, void* pending) {
    HostJob& h = b->jobs[slot];
    LatticeView v;
    v.p = &h.p;
    v.g = make_geom(h.p);
    v.stream = b->stream;
    v.cur = cur;
    v.nxt = nxt;
    v.pending = pending;
    v.phi = nullptr;
    v.cd = h.cd;
    v.cf = h.cf;
    v.shape_set = true;
    v.shape = h.fs;
    return v;
}

// View of a job's current state for export and moments.
LatticeView current_view(lb_batch_t* b, int slot);

// Buffer holding a job's current state.
void* job_current(lb_batch_t* b, int slot) {
    HostJob& h = b->jobs[slot];
    const long long done = std::min(b->gstep, h.last) - h.first;
    const size_t half = job_half(b->storage, (size_t)h.p.nx * h.p.ny * h.p.nz);
    return b->arena_base + h.off + ((done & 1) ? half : 0);
}

LatticeView current_view(lb_batch_t* b, int slot) { return job_view(b, slot, job_current(b, slot), nullptr, nullptr); }

}  // namespace

extern "C" {

int lb_batch_create(int32_t max_jobs, int64_t arena_bytes, int32_t storage, int32_t graph_steps, void* hip_stream,
                    lb_batch_t** out) {
    if (!out) return bfail(LB_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_jobs < 1 || max_jobs > 65536) return bfail(LB_EINVAL, "max_jobs outside 1..65536");
    if (arena_bytes < 4096) return bfail(LB_EINVAL, "arena_bytes too small");
    if (storage < LB_STORE_F64 || storage > LB_STORE_BF16) return bfail(LB_EINVAL, "unknown storage");
    if (graph_steps < 2 || (graph_steps & 1)) return bfail(LB_EINVAL, "graph_steps must be even and >= 2");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return bfail(LB_EDEVICE, "no HIP device");
    lb_batch_t* b = new (std::nothrow) lb_batch_t();
    if (!b) return bfail(LB_ENOMEM, "host allocation failed");
    b->max_jobs = max_jobs;
    b->storage = storage;
    b->graph_steps = graph_steps;
    b->stream = (hipStream_t)hip_stream;
    if (!b->stream) {
        // graph capture needs a stream other than the legacy default stream
        if (hipStreamCreate(&b->stream) != hipSuccess) {
            delete b;
            return bfail(LB_EDEVICE, "hipStreamCreate failed");
        }
        b->own_stream = true;
    }
    b->jobs.resize(max_jobs);
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    // tile shape: the process setting (lb_set_tiles) or the default
    const TileSetting ts = tile_setting(TILE_BATCH, storage);
    b->ty = batch_rows(ts.ty);
    b->tz = ts.tz > 0 ? ts.tz : 32;
    // the tile launch holds as many workgroups as are resident at once (LDS
    // beyond 64 KB needs the opt-in); the assembly launch 8 per CU
    const size_t lds = batch_tile_lds(storage, b->ty);
    int per_cu = 0, per_cu_w = 0;
    const void* kern = batch_tile_kernel_of<false>(storage, b->ty);
    const void* kern_w = batch_tile_kernel_of<true>(storage, b->ty);
    hipError_t he = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (he == hipSuccess) he = hipFuncSetAttribute(kern_w, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (he == hipSuccess) he = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kTX * b->ty, lds);
    if (he == hipSuccess) he = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_w, kern_w, kTX * b->ty, lds);
    // one grid for both variants: as many workgroups as are resident at once for either
    per_cu = std::min(per_cu, per_cu_w);
    if (he != hipSuccess || per_cu < 1) {
        if (b->own_stream) (void)hipStreamDestroy(b->stream);
        delete b;
        return bfail(LB_EDEVICE, std::string("batch tile kernel does not fit a CU: ") + hipGetErrorString(he));
    }
    b->grid = cus * per_cu;
    b->agrid = cus * 8;
    int rc = LB_OK;
    if ((rc = bcheck(hipMalloc((void**)&b->arena_base, (size_t)arena_bytes), "hipMalloc arena")) ||
        (rc = bcheck(hipMalloc(&b->d_jobs, desc_size(storage) * max_jobs), "hipMalloc job table")) ||
        (rc = bcheck(hipMalloc((void**)&b->d_nitems, 3 * sizeof(int)), "hipMalloc counts")) ||
        (rc = bcheck(hipMalloc((void**)&b->d_gstep, sizeof(long long)), "hipMalloc step counter")) ||
        (rc = bcheck(hipMemsetAsync(b->d_jobs, 0, desc_size(storage) * max_jobs, b->stream), "clear job table")) ||
        (rc = bcheck(hipMemsetAsync(b->d_nitems, 0, 3 * sizeof(int), b->stream), "clear counts")) ||
        (rc = bcheck(hipMemsetAsync(b->d_gstep, 0, sizeof(long long), b->stream), "clear counter")) ||
        (rc = upload_items(b))) {
        lb_batch_destroy(b);
        return rc;
    }
    b->arena.reset((size_t)arena_bytes);
    *out = b;
    return LB_OK;
}

int lb_batch_destroy(lb_batch_t* b) {
    if (!b) return bfail(LB_EINVAL, "batch is NULL");
    (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->arena_base) (void)hipFree(b->arena_base);
    if (b->d_jobs) (void)hipFree(b->d_jobs);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_nitems) (void)hipFree(b->d_nitems);
    if (b->d_gstep) (void)hipFree(b->d_gstep);
    if (b->staging) (void)hipFree(b->staging);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return LB_OK;
}

int64_t lb_batch_job_bytes(const lb_params* p) {
    std::string why;
    if (validate_params(p, why) != LB_OK) return -1;
    return (int64_t)((job_bytes(*p) + 511) & ~size_t(511));
}

// Admission: validate, place in the arena, write the initial state and take
// the job's first step (for 16-bit storage from the raw FP32 initial state)
// with the one-read step of a single lattice on the batch's tile boxes: the
// job then enters the batch with its state's phase sums.
static int batch_admit(lb_batch_t* b, const lb_params* params, int64_t steps, int32_t* slot,
                       int (*init)(lb_batch_t*, const LatticeView&, const void*), const void* ctx) {
    if (!b || !params || !slot) return bfail(LB_EINVAL, "NULL argument");
    std::string why;
    if (validate_params(params, why) != LB_OK) return bfail(LB_EINVAL, why);
    if (params->storage != b->storage) return bfail(LB_EINVAL, "job storage differs from the batch storage");
    const int K = params->nc_strength > 0.0 ? params->nc_range : 0;
    if (K + 1 > kBatchH) return bfail(LB_EINVAL, "batched jobs support near-contact ranges up to 2");
    if (make_geom(*params).moving) return bfail(LB_EINVAL, "batched jobs do not support moving walls");
    if (params->model != LB_MODEL_COLOUR_GRADIENT)
        return bfail(LB_EINVAL, "batched jobs use the colour-gradient model");
    {
        // 32-bit byte offsets of the tile kernel's buffer resources
        const uint64_t n = (uint64_t)params->nx * params->ny * params->nz;
        const uint64_t devs = 2 * (uint64_t)Q * dev_stride(n);
        const uint64_t span = b->storage >= LB_STORE_F16
                                  ? (devs > 32 * n ? devs : 32 * n)
                                  : (uint64_t)kResArrays * (b->storage == LB_STORE_F64 ? 8 : 4) * raw_stride(n);
        if (span >= ((uint64_t)1 << 32)) return bfail(LB_EINVAL, "job too large for the batched step");
    }
    if (steps < 0) return bfail(LB_EINVAL, "steps must be >= 0");
    // a 16-bit job's raw FP32 initial state lives in the shared staging area
    // only until its first step (taken here) encodes it into its own buffers
    if (b->storage >= LB_STORE_F16 && steps == 0)
        return bfail(LB_EINVAL, "16-bit batched jobs need steps >= 1");
    int s = -1;
    for (int k = 0; k < b->max_jobs; ++k)
        if (!b->jobs[k].used) {
            s = k;
            break;
        }
    if (s < 0) return bfail(LB_ENOMEM, "no free job slot");
    const size_t N = (size_t)params->nx * params->ny * params->nz;
    const size_t bytes = (job_bytes(*params) + 511) & ~size_t(511);
    size_t off = 0;
    if (!b->arena.alloc(bytes, off)) return bfail(LB_ENOMEM, "arena has no room for this job");
    HostJob& h = b->jobs[s];
    h = HostJob();
    h.p = *params;
    if (h.p.scale_log2 == 0) h.p.scale_log2 = 16;
    h.p.kernel = LB_KERNEL_FUSED;
    h.off = off;
    h.bytes = bytes;
    h.cd = make_coeffs<double>(h.p);
    h.cf = make_coeffs<float>(h.p);
    h.fs = job_shape(b, h.p);
    char* b0 = b->arena_base + off;
    char* b1 = b0 + job_half(b->storage, N);
    char* p0 = b0 + 2 * job_half(b->storage, N);
    const bool split = b->storage >= LB_STORE_F16;
    int rc = ensure_staging(b, (split ? lbm::pop_bytes(LB_STORE_F32, N) : 0) + 5 * N * sizeof(double) + 64);
    long long done = 0;
    if (!rc) {
        LatticeView v = job_view(b, s, b0, b1, split ? b->staging : nullptr);
        v.part_in = p0;
        v.part_out = p0 + job_part(h.p);
        v.part_valid = false;
        rc = init(b, v, ctx);
        if (!rc && steps > 0) {
            rc = launch_step(v, LB_KERNEL_FUSED, nullptr);
            done = 1;
        }
    }
    if (!rc) rc = bcheck(hipStreamSynchronize(b->stream), "sync");
    if (rc) {
        b->arena.release(off, bytes);
        h = HostJob();
        return rc;
    }
    h.used = true;
    h.first = b->gstep - done;
    h.last = h.first + steps;
    rc = upload_desc(b, s);
    if (!rc) rc = upload_items(b);
    if (rc) {
        b->arena.release(off, bytes);
        h = HostJob();
        return rc;
    }
    *slot = s;
    return LB_OK;
}

struct FieldArgs {
    const void *rr, *rb, *u;
    int dtype, on_device;
    size_t N;
};

static int init_from_fields(lb_batch_t* b, const LatticeView& v, const void* ctx) {
    const FieldArgs* a = (const FieldArgs*)ctx;
    const size_t es = a->dtype == LB_DTYPE_F64 ? 8 : 4;
    const void *rr = a->rr, *rb = a->rb, *u = a->u;
    if (!a->on_device) {
        // host fields go through the staging area behind the raw-state region
        char* st = (char*)b->staging + (b->storage >= LB_STORE_F16 ? lbm::pop_bytes(LB_STORE_F32, a->N) : 0);
        int rc = bcheck(hipMemcpyAsync(st, a->rr, a->N * es, hipMemcpyHostToDevice, b->stream), "H2D");
        if (!rc) rc = bcheck(hipMemcpyAsync(st + a->N * es, a->rb, a->N * es, hipMemcpyHostToDevice, b->stream), "H2D");
        if (!rc && a->u) rc = bcheck(hipMemcpyAsync(st + 2 * a->N * es, a->u, 3 * a->N * es, hipMemcpyHostToDevice, b->stream), "H2D");
        if (rc) return rc;
        rr = st;
        rb = st + a->N * es;
        u = a->u ? st + 2 * a->N * es : nullptr;
    }
    return launch_init(v, rr, rb, u, a->dtype);
}

int lb_batch_add(lb_batch_t* b, const lb_params* params, const void* rho_r, const void* rho_b, const void* u,
                 int32_t dtype, int32_t on_device, int64_t steps, int32_t* slot) {
    if (!rho_r || !rho_b) return bfail(LB_EINVAL, "rho_r and rho_b are required");
    if (dtype != LB_DTYPE_F64 && dtype != LB_DTYPE_F32) return bfail(LB_EINVAL, "bad dtype");
    if (!params) return bfail(LB_EINVAL, "params is NULL");
    FieldArgs a{rho_r, rho_b, u, dtype, on_device, (size_t)params->nx * params->ny * params->nz};
    return batch_admit(b, params, steps, slot, init_from_fields, &a);
}

struct DropletArgs {
    const double *cen, *rad;
    int n;
    double width, background, rho0;
    size_t N;
};

static int init_from_droplets(lb_batch_t* b, const LatticeView& v, const void* ctx) {
    const DropletArgs* a = (const DropletArgs*)ctx;
    char* st = (char*)b->staging + (b->storage >= LB_STORE_F16 ? lbm::pop_bytes(LB_STORE_F32, a->N) : 0);
    double* rr = (double*)st;
    double* rb = rr + a->N;
    double* dc = rb + a->N;
    double* dr = dc + 3 * (size_t)a->n;
    int rc = LB_OK;
    if (a->n) rc = bcheck(hipMemcpyAsync(dc, a->cen, 3 * sizeof(double) * a->n, hipMemcpyHostToDevice, b->stream), "H2D");
    if (!rc && a->n) rc = bcheck(hipMemcpyAsync(dr, a->rad, sizeof(double) * a->n, hipMemcpyHostToDevice, b->stream), "H2D");
    if (!rc) rc = launch_droplets(b->stream, v.g, dc, dr, a->n, a->width, a->background, a->rho0, rr, rb);
    if (!rc) rc = launch_init(v, rr, rb, nullptr, LB_DTYPE_F64);
    return rc;
}

int lb_batch_add_droplets(lb_batch_t* b, const lb_params* params, const double* centres, const double* radii,
                          int32_t n, double width, double background, double rho0, int64_t steps, int32_t* slot) {
    if (!params) return bfail(LB_EINVAL, "params is NULL");
    if (n < 0 || (n > 0 && (!centres || !radii))) return bfail(LB_EINVAL, "bad droplet list");
    if (!(width > 0.0) || !(rho0 > 0.0) || !(background >= -1.0 && background <= 1.0))
        return bfail(LB_EINVAL, "width and rho0 must be > 0, background in [-1, 1]");
    const size_t N = (size_t)params->nx * params->ny * params->nz;
    if (b) {
        // room for the fields and the droplet list behind the raw-state region
        int rc = ensure_staging(b, (b->storage >= LB_STORE_F16 ? lbm::pop_bytes(LB_STORE_F32, N) : 0) +
                                       (2 * N + 4 * (size_t)n + 8) * sizeof(double));
        if (rc) return rc;
    }
    DropletArgs a{centres, radii, n, width, background, rho0, N};
    return batch_admit(b, params, steps, slot, init_from_droplets, &a);
}

int lb_batch_remove(lb_batch_t* b, int32_t slot) {
    if (!b || slot < 0 || slot >= b->max_jobs || !b->jobs[slot].used) return bfail(LB_EINVAL, "no job in that slot");
    HostJob& h = b->jobs[slot];
    h.used = false;
    int rc = upload_desc(b, slot);
    if (!rc) rc = upload_items(b);
    b->arena.release(h.off, h.bytes);
    h = HostJob();
    return rc;
}

int lb_batch_step(lb_batch_t* b, int32_t n) {
    if (!b) return bfail(LB_EINVAL, "batch is NULL");
    if (n < 0) return bfail(LB_EINVAL, "n must be >= 0");
    int rc = LB_OK;
    int left = n;
    if (left >= b->graph_steps) {
        rc = ensure_graph(b);
        if (rc) return rc;
        while (left >= b->graph_steps && !rc) {
            rc = bcheck(hipGraphLaunch(b->exec, b->stream), "hipGraphLaunch");
            if (!rc) {
                left -= b->graph_steps;
                b->gstep += b->graph_steps;
            }
        }
    }
    while (left > 0 && !rc) {
        rc = batch_step_once(b);
        if (!rc) {
            --left;
            b->gstep += 1;
        }
    }
    return rc;
}

int64_t lb_batch_job_steps(const lb_batch_t* b, int32_t slot) {
    if (!b || slot < 0 || slot >= b->max_jobs || !b->jobs[slot].used) return -1;
    const HostJob& h = b->jobs[slot];
    return std::min(b->gstep, (long long)h.last) - h.first;
}

int64_t lb_batch_free_bytes(const lb_batch_t* b) { return b ? (int64_t)b->arena.largest() : -1; }

int lb_batch_moments(lb_batch_t* b, int32_t slot, void* rho_r, void* rho_b, void* mom, int32_t dtype,
                     int32_t on_device, double totals[14]) {
    if (!b || slot < 0 || slot >= b->max_jobs || !b->jobs[slot].used) return bfail(LB_EINVAL, "no job in that slot");
    if (dtype != LB_DTYPE_F64 && dtype != LB_DTYPE_F32) return bfail(LB_EINVAL, "bad dtype");
    HostJob& h = b->jobs[slot];
    const size_t N = (size_t)h.p.nx * h.p.ny * h.p.nz;
    const size_t es = dtype == LB_DTYPE_F64 ? 8 : 4;
    LatticeView v = current_view(b, slot);
    int rc = LB_OK;
    if (rho_r || rho_b || mom) {
        if (!on_device) rc = ensure_staging(b, 5 * N * es + 64);
        if (rc) return rc;
        char* st = (char*)b->staging;
        void* o_rr = rho_r ? (on_device ? rho_r : st) : nullptr;
        void* o_rb = rho_b ? (on_device ? rho_b : st + N * es) : nullptr;
        void* o_j = mom ? (on_device ? mom : st + 2 * N * es) : nullptr;
        rc = launch_moments(v, o_rr, o_rb, o_j, dtype);
        if (!rc && !on_device) {
            if (rho_r) rc = bcheck(hipMemcpyAsync(rho_r, o_rr, N * es, hipMemcpyDeviceToHost, b->stream), "D2H");
            if (!rc && rho_b) rc = bcheck(hipMemcpyAsync(rho_b, o_rb, N * es, hipMemcpyDeviceToHost, b->stream), "D2H");
            if (!rc && mom) rc = bcheck(hipMemcpyAsync(mom, o_j, 3 * N * es, hipMemcpyDeviceToHost, b->stream), "D2H");
        }
        if (!rc) rc = bcheck(hipStreamSynchronize(b->stream), "sync");
        if (rc) return rc;
    }
    if (totals) {
        // partials and totals live after the staging fields
        const size_t need = 5 * N * 8 + sizeof(Neu) * NTOT * kTotalsBlocks + 2 * NTOT * sizeof(double) + 512;
        rc = ensure_staging(b, need);
        if (rc) return rc;
        char* base = (char*)b->staging + 5 * N * 8;
        base = (char*)(((uintptr_t)base + 255) & ~uintptr_t(255));
        Neu* partial = (Neu*)base;
        double* dtot = (double*)(base + sizeof(Neu) * NTOT * kTotalsBlocks);
        rc = launch_totals(v, partial, dtot);
        if (!rc) rc = bcheck(hipMemcpyAsync(totals, dtot, sizeof(double) * 2 * NTOT, hipMemcpyDeviceToHost, b->stream), "D2H totals");
        if (!rc) rc = bcheck(hipStreamSynchronize(b->stream), "sync");
    }
    return rc;
}

int lb_batch_get_state(lb_batch_t* b, int32_t slot, void* f, int32_t dtype, int32_t on_device) {
    if (!b || !f || slot < 0 || slot >= b->max_jobs || !b->jobs[slot].used) return bfail(LB_EINVAL, "no job in that slot");
    if (dtype != LB_DTYPE_F64 && dtype != LB_DTYPE_F32) return bfail(LB_EINVAL, "bad dtype");
    HostJob& h = b->jobs[slot];
    const size_t N = (size_t)h.p.nx * h.p.ny * h.p.nz;
    const size_t bytes = 2 * Q * N * (dtype == LB_DTYPE_F64 ? 8 : 4);
    void* out = f;
    int rc = LB_OK;
    if (!on_device) {
        rc = ensure_staging(b, bytes);
        if (rc) return rc;
        out = b->staging;
    }
    LatticeView v = current_view(b, slot);
    rc = launch_export(v, out, dtype);
    if (!rc && !on_device) rc = bcheck(hipMemcpyAsync(f, out, bytes, hipMemcpyDeviceToHost, b->stream), "D2H state");
    if (!rc) rc = bcheck(hipStreamSynchronize(b->stream), "sync");
    return rc;
}

}  // extern "C"
