// Context, geometry cache, tile lists and kernel timing.
#include "common.h"

#include <algorithm>

namespace mmof {

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

bool Geom::same_as(const mmof_stack& s) const {
    if (s.n_seq != n_seq) return false;
    for (int i = 0; i < n_seq; ++i)
        if (s.n_t[i] != n_t[i] || s.ny[i] != ny[i] || s.nx[i] != nx[i]) return false;
    return true;
}

static void build_geom(Geom& g, const mmof_stack* s, hipStream_t st) {
    MMOF_CHECK(s != nullptr, MMOF_ERR_INVALID, "stack is NULL");
    MMOF_CHECK(s->n_seq >= 1, MMOF_ERR_SHAPE, "stack needs n_seq >= 1");
    MMOF_CHECK(s->n_t && s->ny && s->nx, MMOF_ERR_INVALID, "stack arrays are NULL");
    g.n_seq = s->n_seq;
    g.n_t.assign(s->n_t, s->n_t + s->n_seq);
    g.ny.assign(s->ny, s->ny + s->n_seq);
    g.nx.assign(s->nx, s->nx + s->n_seq);
    int64_t off = 0, gx = 0, gy = 0, poff = 0, boff = 0;
    for (int i = 0; i < g.n_seq; ++i) {
        MMOF_CHECK(g.n_t[i] >= 1 && g.ny[i] >= 2 && g.nx[i] >= 2, MMOF_ERR_SHAPE,
                   "sequence " + std::to_string(i) + " needs n_t >= 1, ny >= 2, nx >= 2");
        // (the flow adjoint packs a pixel's two coordinates into 16 bits each)
        MMOF_CHECK(g.ny[i] <= 65535 && g.nx[i] <= 65535, MMOF_ERR_SHAPE, "frame too large (at most 65535 pixels a side)");
        g.seq_off.push_back(off);
        g.max_ny = std::max(g.max_ny, g.ny[i]);
        g.max_nx = std::max(g.max_nx, g.nx[i]);
        for (int t = 0; t < g.n_t[i]; ++t) {
            FrameInfo f{};
            f.off = off;
            f.gx_off = gx;
            f.gy_off = gy;
            f.pair_off = poff;
            f.ny = g.ny[i];
            f.nx = g.nx[i];
            f.t = t;
            f.n_t = g.n_t[i];
            f.seq = i;
            f.blk_off = (int32_t)boff;
            g.frames.push_back(f);
            int64_t np = (int64_t)g.ny[i] * g.nx[i];
            off += np;
            gx += (int64_t)g.ny[i] * (g.nx[i] - 1);
            gy += (int64_t)(g.ny[i] - 1) * g.nx[i];
            if (t + 1 < g.n_t[i]) {
                poff += np;
                boff += (int64_t)((g.ny[i] + 15) / 16) * ((g.nx[i] + 15) / 16);
                MMOF_CHECK(boff < INT32_MAX, MMOF_ERR_SHAPE, "too many frame pairs");
                g.n_pairs += 1;
            }
        }
    }
    g.n = off;
    g.n_frames = (int64_t)g.frames.size();
    g.vec4 = true;
    for (int i = 0; i < g.n_seq; ++i) g.vec4 = g.vec4 && g.nx[i] % 4 == 0;
    g.pair_px = poff;
    g.pair_blocks = boff;
    g.gx_len = gx;
    g.gy_len = gy;
    g.d_frames.ensure(sizeof(FrameInfo) * g.frames.size());
    MMOF_HIP(hipMemcpyAsync(g.d_frames.ptr, g.frames.data(), sizeof(FrameInfo) * g.frames.size(),
                            hipMemcpyHostToDevice, st));
    MMOF_HIP(hipStreamSynchronize(st));
}

const TileList& Geom::tile_list(hipStream_t st, int tw, int th, bool pairs) {
    uint64_t key = ((uint64_t)tw << 33) | ((uint64_t)th << 1) | (pairs ? 1u : 0u);
    auto it = tiles.find(key);
    if (it != tiles.end()) return *it->second;
    std::vector<Tile> host;
    for (int64_t f = 0; f < n_frames; ++f) {
        const FrameInfo& fi = frames[f];
        if (pairs && fi.t + 1 >= fi.n_t) continue;
        for (int y0 = 0; y0 < fi.ny; y0 += th)
            for (int x0 = 0; x0 < fi.nx; x0 += tw) host.push_back(Tile{(int32_t)f, y0, x0, 0});
    }
    std::unique_ptr<TileList> tl(new TileList());
    tl->count = (int64_t)host.size();
    tl->buf.ensure(sizeof(Tile) * std::max<size_t>(host.size(), 1));
    if (!host.empty()) {
        MMOF_HIP(hipMemcpyAsync(tl->buf.ptr, host.data(), sizeof(Tile) * host.size(), hipMemcpyHostToDevice, st));
        MMOF_HIP(hipStreamSynchronize(st));
    }
    MMOF_CHECK(tl->count < (int64_t)INT32_MAX, MMOF_ERR_SHAPE, "too many tiles");
    auto& ref = *tl;
    tiles[key] = std::move(tl);
    return ref;
}

const TileList& Geom::adj_tile_list(hipStream_t st, int tw, int th) {
    const uint64_t key = ((uint64_t)tw << 32) | (uint64_t)th;
    auto it = adj_tiles.find(key);
    if (it != adj_tiles.end()) return *it->second;
    std::vector<AdjTile> host;
    for (int64_t f = 0; f < n_frames; ++f) {
        const FrameInfo& fi = frames[f];
        const int64_t po = fi.t + 1 < fi.n_t ? fi.pair_off : -1;
        const int64_t pp = fi.t >= 1 ? frames[f - 1].pair_off : -1;
        for (int y0 = 0; y0 < fi.ny; y0 += th)
            for (int x0 = 0; x0 < fi.nx; x0 += tw) host.push_back(AdjTile{fi.off, po, pp, fi.nx, fi.ny, x0, y0});
    }
    std::unique_ptr<TileList> tl(new TileList());
    tl->count = (int64_t)host.size();
    tl->buf.ensure(sizeof(AdjTile) * std::max<size_t>(host.size(), 1));
    if (!host.empty()) {
        MMOF_HIP(hipMemcpyAsync(tl->buf.ptr, host.data(), sizeof(AdjTile) * host.size(), hipMemcpyHostToDevice, st));
        MMOF_HIP(hipStreamSynchronize(st));
    }
    MMOF_CHECK(tl->count < (int64_t)INT32_MAX, MMOF_ERR_SHAPE, "too many tiles");
    auto& ref = *tl;
    adj_tiles[key] = std::move(tl);
    return ref;
}

std::unique_ptr<Geom> make_geom(const mmof_stack* s, hipStream_t st) {
    std::unique_ptr<Geom> g(new Geom());
    build_geom(*g, s, st);
    return g;
}

Geom& Ctx::geom(const mmof_stack* s) {
    MMOF_CHECK(s != nullptr, MMOF_ERR_INVALID, "stack is NULL");
    // most recently used last, so that a call holding the geometry it looked up first can
    // look up a second one without evicting the first
    for (size_t i = 0; i < geoms.size(); ++i)
        if (geoms[i]->same_as(*s)) {
            std::unique_ptr<Geom> hit = std::move(geoms[i]);
            geoms.erase(geoms.begin() + (std::ptrdiff_t)i);
            geoms.push_back(std::move(hit));
            return *geoms.back();
        }
    std::unique_ptr<Geom> g(new Geom());
    build_geom(*g, s, stream);
    if (geoms.size() >= 16) geoms.erase(geoms.begin());
    geoms.push_back(std::move(g));
    return *geoms.back();
}

Ctx::~Ctx() {
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    if (pinned_buf) (void)hipHostFree(pinned_buf);
    for (auto& e : timer.events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
}

void* Ctx::pinned(size_t bytes) {
    if (bytes <= pinned_bytes && pinned_buf) return pinned_buf;
    if (pinned_buf) (void)hipHostFree(pinned_buf);
    pinned_buf = nullptr;
    pinned_bytes = 0;
    MMOF_HIP(hipHostMalloc(&pinned_buf, bytes, hipHostMallocDefault));
    pinned_bytes = bytes;
    return pinned_buf;
}

void Ctx::time_begin(const char*, hipEvent_t* ev) {
    hipEvent_t a, b;
    MMOF_HIP(hipEventCreate(&a));
    MMOF_HIP(hipEventCreate(&b));
    MMOF_HIP(hipEventRecord(a, stream));
    timer.events.push_back({a, b});
    *ev = b;
}

void Ctx::time_end(const char*, hipEvent_t ev) { (void)hipEventRecord(ev, stream); }

}  // namespace mmof
