// Internal runtime of the MMGKS-OF library: context, geometry, tiles, errors.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <initializer_list>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/mmof.h"

namespace mmof {

// ----------------------------------------------------------------------------- errors

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define MMOF_HIP(call)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::mmof::Error(MMOF_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define MMOF_CHECK(cond, code, msg)                      \
    do {                                                 \
        if (!(cond)) throw ::mmof::Error((code), (msg)); \
    } while (0)

// Launch + error check (launch errors are reported synchronously by hipGetLastError).
#define MMOF_LAUNCH_CHECK() MMOF_HIP(hipGetLastError())

// ----------------------------------------------------------------------------- device tables

// One frame of a packed stack.
struct FrameInfo {
    int64_t off;       // pixel offset of the frame in the stack
    int64_t gx_off;    // offset of its gx block ([ny][nx-1])
    int64_t gy_off;    // offset of its gy block ([ny-1][nx])
    int64_t pair_off;  // pixel offset of pair (t, t+1) in pair arrays (valid if t < n_t-1)
    int32_t ny, nx;
    int32_t t, n_t;
    int32_t seq;
    int32_t blk_off;   // pairs: offset of the frame's 16 x 16 blocks in per-block arrays
};

// A rectangular work tile of one frame (or one pair: frame = first frame of the pair).
struct Tile {
    int32_t frame;
    int32_t y0, x0;
    int32_t pad;
};

// A tile of one frame with what the flow adjoint needs of the frame and its neighbour,
// so a workgroup finds everything in one load.
struct alignas(16) AdjTile {
    int64_t off;  // pixel offset of the frame
    int64_t po;   // pixel offset (in pair arrays) of pair (t, t+1); -1 for the last frame
    int64_t pp;   // pixel offset of pair (t-1, t); -1 for the first frame
    int32_t nx, ny;
    int32_t x0, y0;
};

// ----------------------------------------------------------------------------- host objects

struct DeviceBuffer {
    void* ptr = nullptr;
    size_t bytes = 0;
    DeviceBuffer() = default;
    DeviceBuffer(const DeviceBuffer&) = delete;
    DeviceBuffer& operator=(const DeviceBuffer&) = delete;
    ~DeviceBuffer() { release(); }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    // Grows (never shrinks); contents are not preserved.
    void* ensure(size_t nbytes) {
        if (nbytes <= bytes && ptr) return ptr;
        release();
        size_t want = nbytes ? nbytes : 256;
        hipError_t e = hipMalloc(&ptr, want);
        if (e != hipSuccess) {
            ptr = nullptr;
            throw Error(MMOF_ERR_OOM, "hipMalloc of " + std::to_string(want) + " bytes failed");
        }
        bytes = want;
        return ptr;
    }
    template <class T> T* as() const { return static_cast<T*>(ptr); }
};

struct TileList {
    DeviceBuffer buf;
    int64_t count = 0;
};

// Output tile of a stencil kernel: tw x th pixels per workgroup; persistent: the grid is a
// few workgroups per CU that loop over the tile list.
struct TileShape {
    int tw, th, persistent;
};

struct Geom {
    std::vector<int32_t> n_t, ny, nx;
    int32_t n_seq = 0;
    int64_t n = 0;          // pixels
    int64_t n_frames = 0;
    int64_t n_pairs = 0;    // frame pairs
    int64_t pair_px = 0;    // pixels over all pairs
    int64_t pair_blocks = 0;  // 16 x 16 blocks (partial ones included) over all pairs
    int64_t gx_len = 0, gy_len = 0;
    int32_t max_ny = 0, max_nx = 0;
    // every frame width is a multiple of 4, so frame, pair and row starts (and those of the
    // gy blocks) fall on 4-element boundaries: the stencil kernels may move 4 pixels at once
    bool vec4 = false;
    std::vector<FrameInfo> frames;       // host copy
    std::vector<int64_t> seq_off;        // pixel offset per sequence
    DeviceBuffer d_frames;               // FrameInfo[n_frames]
    std::map<uint64_t, std::unique_ptr<TileList>> tiles;  // (tw, th, pairs) -> list
    std::map<uint64_t, std::unique_ptr<TileList>> adj_tiles;  // (tw, th) -> AdjTile list
    // Tile-shape candidate chosen by the autotuner per "kernel/dtype".  Untuned kernels use
    // candidate 0 (tiles of 1024 outputs) on frames of at least 512 x 512 pixels and
    // `small` (tiles of 256 outputs, more workgroups) on smaller frames.
    std::map<std::string, int> tuned;
    int choice(const char* kernel, int dt, int small = 0) const {
        auto it = tuned.find(std::string(kernel) + (dt == MMOF_F32 ? "/f32" : "/f64"));
        if (it != tuned.end()) return it->second;
        return (int64_t)max_nx * max_ny >= 512 * 512 ? 0 : small;
    }

    bool same_as(const mmof_stack& s) const;
    const TileList& tile_list(hipStream_t st, int tw, int th, bool pairs);
    const TileList& adj_tile_list(hipStream_t st, int tw, int th);
    const FrameInfo* dframes() const { return d_frames.as<FrameInfo>(); }
};

std::unique_ptr<Geom> make_geom(const mmof_stack* s, hipStream_t st);

struct KernelTimer {
    std::string name;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    int64_t launches = 0;
    double total_ms = 0.0;
    double bytes = 0.0, flops = 0.0;  // algorithmic work of the timed launches
};

// An instantiated HIP graph of a launch sequence and the operator-application counts one
// replay adds to a solve report.
struct CachedGraph {
    hipGraphExec_t exec = nullptr;
    int64_t dA = 0, dAt = 0, dTheta = 0, dThetaT = 0, dL = 0;
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string last_error;
    std::vector<std::unique_ptr<Geom>> geoms;   // small cache keyed by content
    std::map<std::string, std::unique_ptr<DeviceBuffer>> ws;  // named workspaces
    KernelTimer timer;
    int cu_count = 256;
    // private stream the launch sequences of a solve are captured on (capture is not possible on the legacy
    // default stream); the graphs are launched on `stream`
    hipStream_t capture_stream = nullptr;
    bool capturing = false;  // launches are being recorded into a graph (no event timing)
    void* pinned_buf = nullptr;
    size_t pinned_bytes = 0;
    ~Ctx();
    // Pinned host staging buffer (grows; contents not preserved).
    void* pinned(size_t bytes);

    Geom& geom(const mmof_stack* s);
    void* work(const std::string& name, size_t bytes) {
        auto& p = ws[name];
        if (!p) p.reset(new DeviceBuffer());
        return p->ensure(bytes);
    }
    // Device memory that work(name, bytes) would take beyond what the buffer holds now (a
    // growing buffer is freed before the larger one is allocated, so only the difference is new).
    size_t work_growth(const std::string& name, size_t bytes) const {
        auto it = ws.find(name);
        const size_t have = (it != ws.end() && it->second) ? it->second->bytes : 0;
        return bytes > have ? bytes - have : 0;
    }
    // Event-timing hooks around launches of a named kernel.
    bool timing(const char* kname) const { return !capturing && !timer.name.empty() && timer.name == kname; }
    void time_begin(const char* kname, hipEvent_t* ev);
    void time_end(const char* kname, hipEvent_t ev);
};

struct Plan {
    Ctx* ctx = nullptr;
    int kind = 0;  // 0 radon (parallel beam), 1 blur, 2 fan beam
    std::unique_ptr<Geom> geom_own;  // the plan's own copy of its stack geometry
    Geom* geom = nullptr;
    int64_t n = 0, m = 0;
    // radon
    std::vector<int32_t> n_ang, n_bins;
    double radon_flops = 0.0;       // 2 hat weights x (multiply + add) per pixel and angle
    std::vector<int64_t> sino_off;  // per frame, offset of its sinogram
    DeviceBuffer d_trig;            // float2/double2 per (frame, angle): cos, sin  (double)
    DeviceBuffer d_rinfo;           // RadonFrame[n_frames]
    DeviceBuffer d_rays[4];         // ray tiles of the forward projector (angle groups 1, 2, 4, 8)
    DeviceBuffer d_tiles_a;         // pixel tiles of the back-projector
    DeviceBuffer d_tiles_b;         // 32x32 tiles of the frame transpose
    bool tr_vec = false;            // every frame side and offset a multiple of 4 (vector transpose)
    int64_t n_rays[4] = {0, 0, 0, 0}, n_tiles_a = 0, n_tiles_b = 0;
    // fan beam: source-to-centre and source-to-detector distances, bin width (pixel units)
    double fan_dso = 0.0, fan_dsd = 0.0, fan_du = 0.0;
    DeviceBuffer d_fanrays;         // double4 per ray (sinogram layout): line and path length
    // blur
    int ksize = 9;
    double sigma = 2.0;
    DeviceBuffer d_k1;              // 1-D factor (double) [ksize]
    // launch sequences of solves on this plan captured as graphs, keyed by every pointer and
    // choice their launches depend on; they die with the plan (and its tile lists)
    std::map<std::string, CachedGraph> graphs;
    std::map<std::string, int> graph_seen;
    // geometries of the frames reduced for the flow (by factor), owned by the plan so that
    // captured graphs keep valid tile lists
    std::map<int, std::unique_ptr<Geom>> reduced;
    Plan() = default;
    Plan(const Plan&) = delete;
    Plan& operator=(const Plan&) = delete;
    ~Plan() {
        for (auto& g : graphs)
            if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
    }
};

// Scoped kernel timer: records events around a launch when the kernel is selected.
struct ScopedTime {
    Ctx* c;
    const char* name;
    hipEvent_t ev = nullptr;
    // bytes / flops: the launch's algorithmic work (each input read once, each output written
    // once; the arithmetic the method needs), accumulated while the kernel is being timed
    // (c == nullptr: never timed)
    ScopedTime(Ctx* c_, const char* n, double bytes = 0.0, double flops = 0.0) : c(c_), name(n) {
        if (c && c->timing(name)) {
            c->time_begin(name, &ev);
            c->timer.bytes += bytes;
            c->timer.flops += flops;
        }
    }
    ~ScopedTime() {
        if (ev) c->time_end(name, ev);
    }
};

// dtype dispatch helper
template <class F>
void dispatch(int dt, F&& f) {
    if (dt == MMOF_F32)
        f(float{});
    else if (dt == MMOF_F64)
        f(double{});
    else
        throw Error(MMOF_ERR_DTYPE, "unsupported dtype " + std::to_string(dt));
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// All pointers aligned to `bytes` (null pointers pass).
inline bool aligned_to(size_t bytes, std::initializer_list<const void*> ptrs) {
    for (const void* p : ptrs)
        if (reinterpret_cast<uintptr_t>(p) % bytes) return false;
    return true;
}

// Grid for a 1-D grid-stride launch.
inline dim3 grid_for(int64_t n, int block, int cap = 65536) {
    int64_t g = cdiv(n, block);
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return dim3((unsigned)g);
}

}  // namespace mmof

// The opaque handles of the ABI.
struct mmof_ctx_s : mmof::Ctx {};
struct mmof_plan_s : mmof::Plan {};
