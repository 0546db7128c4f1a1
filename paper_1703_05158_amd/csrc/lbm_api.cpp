// Host side of liblbm: argument validation, device memory, state machine and
// the per-step launch sequence.  Every entry point returns an lbm_status and
// never throws across the C ABI.
#include "lbm.h"
#include "lbm_device.h"
#include "lbm_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

using namespace lbm;

struct lbm_ctx {
    lbm_config cfg{};
    hipStream_t stream = nullptr;
    int N = 0;
    int Ns = 0;                        // stride between the 19 direction arrays
    int sbytes = 4;
    void *pop[2] = {nullptr, nullptr};
    int cur = 0;                       // pop[cur] holds the current (post-collision) state
    uint16_t *own = nullptr;
    uint8_t *wall_map = nullptr;
    double *tab[2] = {nullptr, nullptr};
    int ts = 0;                        // tab[ts]: bodies of the current state's geometry
    int nb_state = 0, nb_next = 0;
    bool dirty = false;                // tab[1-ts] set since the last step / init
    double *walls = nullptr;
    double *wrec = nullptr;            // max_walls * kBodyStride: the walls as link records {ref, U, 0, 0}
    int n_walls = 0;
    double *acc = nullptr;             // (max_bodies + max_walls) * 6: forces of the last step
    // fused step: fixed-point force sums, (max_bodies + max_walls * kWallRep) * 6
    // each; the steps alternate between the two buffers.  The sums of the last
    // step stay pending until lbm_get_forces[_device] or the next fused step
    // turns them into acc.
    unsigned long long *fsum[2] = {nullptr, nullptr};
    int fcur = 0;                      // buffer of the next fused step
    bool fpending = false;             // the last step's sums are not yet in acc
    FinishArgs pend{};                 // where they are: buffer, wall base, counts
    unsigned long long *static_fix = nullptr; // this device's static sums of lbm_step_noalloc
    hipError_t static_fix_err = hipSuccess;   // why static_fix is null
    int path = LBM_PATH_FUSED;         // lbm_step_path
    uint64_t geom_gen = 0;             // bumped whenever the geometry, the body force or the state is replaced
    int tile = kTile64x2x2;            // TileShape of the step kernel
    int ntx = 0, nty = 0, ntz = 0, n_tiles = 0;
    // wall links (fixed while the walls are): fluid nodes per (wall, direction),
    // workgroup chunks, per-chunk sums, each wall's range of chunks
    uint32_t *wl_node = nullptr;
    int *wl_blk = nullptr, *wl_wblk = nullptr;
    double *wl_part = nullptr;
    int n_wblk = 0;
    int64_t wl_bytes = 0;
    std::vector<uint8_t> wall_host;    // host copy of the wall map
    // inflow plane fed by a virtual cylinder (Sec. 2.6); zieb_z < 0: none
    int zieb_z = -1;
    double zieb_area = 0.0, zieb_volume = 0.0, zieb_vp = 0.0;
    double *zstate = nullptr;          // ZiebState on the device
    double *zpart = nullptr;           // kZiebMaxBlocks * 3 doubles, then a uint32 counter: the plane reduction
    int *flag = nullptr;
    int *flag_host = nullptr;
    double *scratch = nullptr;         // 4N doubles, export/import staging (lazy)
    double *pinned = nullptr;          // max_bodies * 10 doubles, set_bodies staging
    double *forces_pin = nullptr;      // (max_bodies + max_walls) * 6 doubles, get_forces staging
    int *order = nullptr;              // max_bodies: sphere order of the link pass (Morton order of the centres)
    int *order_pin = nullptr;          // its host staging
    int n_order = 0;                   // body count the order was made for (0: none)
    int order_age = 0;                 // host body tables staged since the order was made
    hipEvent_t stage_evt = nullptr;
    bool initialized = false;
    int steps_done = 0;
    int64_t device_bytes = 0;
    bool prof = false;
    int prof_every = 1;                // profile every prof_every-th step
    int64_t prof_n = 0;                // steps since profiling was switched on
    // profiling: per step, events at the start, after the geometry update,
    // after the link pass (split path), after the step kernel and after the
    // force finish; events come from a pool that lives as long as the handle
    std::vector<std::array<hipEvent_t, 4>> prof_ev;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::string err;
};

namespace {

const char *kNullHandle = "null lbm_handle";

lbm_status fail(lbm_ctx *h, lbm_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    return st;
}

#define HIP_TRY(h, expr)                                                                         \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail((h), e_ == hipErrorOutOfMemory ? LBM_ERR_OOM : LBM_ERR_HIP, "%s: %s (%s)", \
                        #expr, hipGetErrorString(e_), hipGetErrorName(e_));                      \
    } while (0)

bool finite_all(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// A failed runtime call leaves its code as the last error, which the next
// kernel launch would report as its own: cleared, the code passed on.
hipError_t cleared(hipError_t e)
{
    if (e != hipSuccess) (void)hipGetLastError();
    return e;
}

template <typename T>
hipError_t dalloc(lbm_ctx *h, T **p, size_t bytes)
{
    hipError_t e = cleared(hipMalloc((void **)p, bytes ? bytes : 16));
    if (e == hipSuccess) h->device_bytes += (int64_t)bytes;
    return e;
}

GeomArgs geom(const lbm_ctx *h)
{
    GeomArgs g{};
    g.nx = h->cfg.nx;
    g.ny = h->cfg.ny;
    g.nz = h->cfg.nz;
    g.N = h->N;
    g.Ns = h->Ns;
    g.n_walls = h->n_walls;
    g.bodies = h->tab[h->ts];
    g.nb = h->nb_state;
    g.own = h->own;
    g.pop = h->pop[h->cur];
    g.rho0 = (float)h->cfg.rho0;
    return g;
}

void set_tile_shape(lbm_ctx *h, int shape)
{
    h->tile = shape;
    h->ntx = (h->cfg.nx + kTileDims[shape][0] - 1) / kTileDims[shape][0];
    h->nty = (h->cfg.ny + kTileDims[shape][1] - 1) / kTileDims[shape][1];
    h->ntz = (h->cfg.nz + kTileDims[shape][2] - 1) / kTileDims[shape][2];
    h->n_tiles = h->ntx * h->nty * h->ntz;
}

// Arguments of the step kernel (src/dst of the current state) and of the
// link pass (pop of the current state, bodies of the current geometry).
StepArgs step_args(const lbm_ctx *h)
{
    const lbm_config &c = h->cfg;
    StepArgs a{};
    a.nx = c.nx;
    a.ny = c.ny;
    a.nz = c.nz;
    a.N = h->N;
    a.Ns = h->Ns;
    a.tile = h->tile;
    a.ntx = h->ntx;
    a.nty = h->nty;
    a.ntz = h->ntz;
    a.n_tiles = h->n_tiles;
    a.tau0 = (float)c.tau0;
    a.smag_k = (float)(18.0 * std::sqrt(2.0) * c.smag_c * c.smag_c);
    a.rho0 = (float)c.rho0;
    a.fx = (float)c.body_force[0];
    a.fy = (float)c.body_force[1];
    a.fz = (float)c.body_force[2];
    a.own = h->own;
    a.flag = c.nan_guard_every > 0 ? h->flag : nullptr;
    a.src = h->pop[h->cur];
    a.dst = h->pop[1 - h->cur];
    a.zieb_z = h->zieb_z;
    a.zieb_state = h->zstate;
    return a;
}

ZiebArgs zieb_args(const lbm_ctx *h)
{
    ZiebArgs z{};
    z.nx = h->cfg.nx;
    z.ny = h->cfg.ny;
    z.nz = h->cfg.nz;
    z.N = h->N;
    z.Ns = h->Ns;
    z.z = h->zieb_z;
    z.rho0 = (float)h->cfg.rho0;
    z.fz = (float)h->cfg.body_force[2];
    z.area = h->zieb_area;
    z.volume = h->zieb_volume;
    z.vp = h->zieb_vp;
    z.own = h->own;
    z.pop = h->pop[h->cur];
    z.state = h->zstate;
    z.part = h->zpart;
    z.done = reinterpret_cast<unsigned int *>(h->zpart + 3 * kZiebMaxBlocks);
    return z;
}

LinkArgs link_args(const lbm_ctx *h)
{
    const lbm_config &c = h->cfg;
    LinkArgs la{};
    la.nx = c.nx;
    la.ny = c.ny;
    la.nz = c.nz;
    la.Ns = h->Ns;
    la.halfway = c.bb_mode == LBM_BB_HALFWAY;
    la.rho0 = (float)c.rho0;
    la.own = h->own;
    la.walls = h->walls;
    la.wrec = h->wrec;
    la.wl_node = h->wl_node;
    la.wl_blk = h->wl_blk;
    la.wl_wblk = h->wl_wblk;
    la.wl_part = h->wl_part;
    la.out = h->acc;
    la.n_walls = h->n_walls;
    la.n_wblk = h->n_walls > 0 ? h->n_wblk : 0;
    la.nb = h->nb_state;
    la.order = h->n_order == h->nb_state ? h->order : nullptr;
    la.bodies = h->tab[h->ts];
    la.pop = h->pop[h->cur];
    return la;
}

size_t fsum_entries(const lbm_config &c) { return 6 * ((size_t)c.max_bodies + (size_t)c.max_walls * kWallRep); }

FusedArgs fused_args(const lbm_ctx *h)
{
    FusedArgs f{};
    f.s = step_args(h);
    f.n_walls = h->n_walls;
    f.nb = h->nb_state;
    f.halfway = h->cfg.bb_mode == LBM_BB_HALFWAY;
    f.bodies = h->tab[h->ts];
    f.wrec = h->wrec;
    f.fsum = h->fsum[h->fcur];
    f.wall_base = h->cfg.max_bodies;
    return f;
}

// The pending sums of the last fused step, to be turned into acc.
FinishArgs pending_finish(const lbm_ctx *h)
{
    FinishArgs fa = h->pend;
    fa.out = h->acc;
    fa.out2 = nullptr;
    return fa;
}

// Turn pending force sums into acc (and a copy in out2, if given).
lbm_status finish_forces(lbm_ctx *h, double *out2)
{
    if (!h->fpending) return LBM_OK;
    FinishArgs fa = pending_finish(h);
    fa.out2 = out2;
    HIP_TRY(h, launch_finish(fa, h->stream));
    h->fpending = false;
    return LBM_OK;
}

// Clear both force-sum buffers and any pending step.
lbm_status reset_sums(lbm_ctx *h)
{
    for (int k = 0; k < 2; ++k) HIP_TRY(h, launch_zero_fix(h->fsum[k], (int)fsum_entries(h->cfg), h->stream));
    h->fpending = false;
    h->fcur = 0;
    return LBM_OK;
}


// An event of the handle's pool for the profile of one step.
hipError_t prof_event(lbm_ctx *h, hipEvent_t *e)
{
    if (h->ev_used == h->ev_pool.size()) {
        hipEvent_t ne = nullptr;
        const hipError_t r = hipEventCreate(&ne);
        if (r != hipSuccess) return r;
        h->ev_pool.push_back(ne);
    }
    *e = h->ev_pool[h->ev_used++];
    return hipSuccess;
}

hipError_t prof_mark(lbm_ctx *h, hipEvent_t *e)
{
    const hipError_t r = prof_event(h, e);
    return r != hipSuccess ? r : hipEventRecord(*e, h->stream);
}

// The NaN guard's flag cleared on the handle's stream (after a state change).
lbm_status clear_flag(lbm_ctx *h)
{
    HIP_TRY(h, hipMemsetAsync(h->flag, 0, sizeof(int), h->stream));
    return LBM_OK;
}

// The wall table (host, [n][kWallStride] = U, ref) as link records
// {ref, U, Omega = 0, R = 0} on the device.
lbm_status upload_wall_records(lbm_ctx *h, const double *wt, int n)
{
    std::vector<double> rec((size_t)kBodyStride * std::max(n, 1), 0.0);
    for (int w = 0; w < n; ++w)
        for (int a = 0; a < 3; ++a) {
            rec[(size_t)w * kBodyStride + a] = wt[(size_t)w * kWallStride + 3 + a];
            rec[(size_t)w * kBodyStride + 3 + a] = wt[(size_t)w * kWallStride + a];
        }
    HIP_TRY(h, hipMemcpyAsync(h->wrec, rec.data(), sizeof(double) * rec.size(), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

// Rebuild the whole owner map: walls, then the spheres of tab[ts].
lbm_status rasterize_full(lbm_ctx *h)
{
    GeomArgs g = geom(h);
    g.bodies2 = g.bodies;  // stamp only
    g.nb2 = g.nb;
    g.nb = 0;
    HIP_TRY(h, launch_walls_init(h->wall_map, h->own, h->N, h->stream));
    HIP_TRY(h, launch_geometry(h->cfg.storage, g, h->stream));
    return LBM_OK;
}

// Move from the geometry of tab[ts] to that of tab[1-ts] (bodies set since
// the last step), refilling uncovered nodes in the current population buffer.
lbm_status rasterize_update(lbm_ctx *h)
{
    GeomArgs g = geom(h);
    g.bodies2 = h->tab[1 - h->ts];
    g.nb2 = h->nb_next;
    HIP_TRY(h, launch_geometry(h->cfg.storage, g, h->stream));
    h->ts = 1 - h->ts;
    h->nb_state = h->nb_next;
    h->dirty = false;
    h->geom_gen++;
    return LBM_OK;
}

// Direction arrays start at staggered offsets: with a power-of-two node count
// all 38 read/write streams of the step would otherwise sit at addresses
// congruent modulo a large power of two.
int pop_stride(int N) { return ((N + 63) / 64) * 64 + 1088; }

lbm_status check_ready(lbm_ctx *h)
{
    if (!h->initialized) return fail(h, LBM_ERR_STATE, "lbm_init_fields has not been called");
    return LBM_OK;
}

lbm_status ensure_scratch(lbm_ctx *h)
{
    if (!h->scratch) HIP_TRY(h, dalloc(h, &h->scratch, sizeof(double) * (size_t)h->N * 4));
    return LBM_OK;
}

// Copy on the handle's stream and wait for it.
lbm_status copy_sync(lbm_ctx *h, void *dst, const void *src, size_t bytes, hipMemcpyKind kind)
{
    if (bytes == 0) return LBM_OK;
    HIP_TRY(h, hipMemcpyAsync(dst, src, bytes, kind, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

// gfx target of the current device ("gfx950"), the key prefix of the
// tile-shape cache.
std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t p{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string s = p.gcnArchName;
    const size_t c = s.find(':');
    return c == std::string::npos ? s : s.substr(0, c);
}

// The tile-shape cache: a flat JSON object of string keys and integer values.
std::map<std::string, int> read_cache(const char *path)
{
    std::map<std::string, int> m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    size_t i = 0;
    while ((i = t.find('"', i)) != std::string::npos) {
        const size_t j = t.find('"', i + 1);
        if (j == std::string::npos) break;
        const size_t c = t.find(':', j);
        if (c == std::string::npos) break;
        char *e = nullptr;
        const long v = std::strtol(t.c_str() + c + 1, &e, 10);
        if (e == t.c_str() + c + 1) break;
        m[t.substr(i + 1, j - i - 1)] = (int)v;
        i = (size_t)(e - t.c_str());
    }
    return m;
}

bool write_cache(const char *path, const std::map<std::string, int> &m)
{
    std::ofstream f(path);
    if (!f) return false;
    f << "{\n";
    size_t k = 0;
    for (const auto &kv : m) f << "  \"" << kv.first << "\": " << kv.second << (++k < m.size() ? ",\n" : "\n");
    f << "}\n";
    return (bool)f;
}

struct EventPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t create()
    {
        hipError_t e = hipEventCreate(&e0);
        return e == hipSuccess ? hipEventCreate(&e1) : e;
    }
    ~EventPair()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

#define TRY(expr)                        \
    do {                                 \
        lbm_status st_ = (expr);         \
        if (st_ != LBM_OK) return st_;   \
    } while (0)

void free_wall_links(lbm_ctx *h)
{
    void *p[] = {h->wl_node, h->wl_blk, h->wl_wblk, h->wl_part};
    for (void *q : p)
        if (q) (void)hipFree(q);
    h->wl_node = nullptr;
    h->wl_blk = h->wl_wblk = nullptr;
    h->wl_part = nullptr;
    h->n_wblk = 0;
    h->device_bytes -= h->wl_bytes;
    h->wl_bytes = 0;
}

// List the wall links of a wall map (host array, ids 1..n_walls, 0 = none):
// every fluid-side node x with the wall voxel x - c_I, grouped by wall and
// direction I, cut into chunks of kWallChunk links.
lbm_status build_wall_links(lbm_ctx *h, const uint8_t *wall, int n_walls)
{
    if (n_walls < 0 || n_walls > h->cfg.max_walls) return fail(h, LBM_ERR_ARG, "n_walls %d out of range", n_walls);
    for (int n = 0; n < h->N; ++n)
        if (wall[n] > n_walls) return fail(h, LBM_ERR_ARG, "wall id %d at node %d exceeds n_walls", wall[n], n);
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    free_wall_links(h);
    const int nx = h->cfg.nx, ny = h->cfg.ny, nz = h->cfg.nz;
    std::vector<std::vector<uint32_t>> seg((size_t)n_walls * (kQ - 1));
    if (n_walls > 0) {
        auto wrap = [](int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); };
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const size_t n = (size_t)x + (size_t)nx * (y + (size_t)ny * z);
                    if (wall[n]) continue;
                    for (int i = 1; i < kQ; ++i) {
                        // links of the inflow plane into the removed domain are not walls
                        if (z == h->zieb_z && dev::CZ[i] == 1) continue;
                        const size_t s = (size_t)wrap(x - dev::CX[i], nx) +
                                         (size_t)nx * (wrap(y - dev::CY[i], ny) + (size_t)ny * wrap(z - dev::CZ[i], nz));
                        const int w = wall[s];
                        if (w) seg[(size_t)(w - 1) * (kQ - 1) + (i - 1)].push_back((uint32_t)n);
                    }
                }
    }
    std::vector<uint32_t> nodes;
    std::vector<int> blk, wblk(1, 0);
    for (int w = 0; w < n_walls; ++w) {
        for (int i = 1; i < kQ; ++i) {
            const int sg = w * (kQ - 1) + (i - 1);
            const std::vector<uint32_t> &v = seg[sg];
            for (size_t c = 0; c < v.size(); c += kWallChunk) {
                blk.push_back(sg);
                blk.push_back((int)(nodes.size() + c));
                blk.push_back((int)(nodes.size() + std::min(v.size(), c + kWallChunk)));
            }
            nodes.insert(nodes.end(), v.begin(), v.end());
        }
        wblk.push_back((int)(blk.size() / 3));
    }
    const int n_wblk = (int)(blk.size() / 3);
    const int64_t before = h->device_bytes;
    const bool ok = dalloc(h, &h->wl_node, sizeof(uint32_t) * nodes.size()) == hipSuccess &&
                    dalloc(h, &h->wl_blk, sizeof(int) * blk.size()) == hipSuccess &&
                    dalloc(h, &h->wl_wblk, sizeof(int) * wblk.size()) == hipSuccess &&
                    dalloc(h, &h->wl_part, sizeof(double) * 6 * (size_t)n_wblk) == hipSuccess;
    h->wl_bytes = h->device_bytes - before;
    if (!ok) {
        // nothing half-made is left for a link pass to read
        free_wall_links(h);
        return fail(h, LBM_ERR_OOM, "no device memory for the wall links");
    }
    h->n_wblk = n_wblk;
    TRY(copy_sync(h, h->wl_node, nodes.data(), sizeof(uint32_t) * nodes.size(), hipMemcpyHostToDevice));
    TRY(copy_sync(h, h->wl_blk, blk.data(), sizeof(int) * blk.size(), hipMemcpyHostToDevice));
    TRY(copy_sync(h, h->wl_wblk, wblk.data(), sizeof(int) * wblk.size(), hipMemcpyHostToDevice));
    return LBM_OK;
}

}  // namespace

extern "C" {

int32_t lbm_version(void) { return 10300; }

const char *lbm_last_error(lbm_handle h) { return h ? h->err.c_str() : kNullHandle; }

lbm_status lbm_create(const lbm_config *cfg, lbm_handle *out)
{
    if (!cfg || !out) return LBM_ERR_ARG;
    const lbm_config &c = *cfg;
    if (c.nx < 1 || c.ny < 1 || c.nz < 1) return LBM_ERR_ARG;
    const long long N = (long long)c.nx * c.ny * c.nz;
    if (N > (long long)0x7fffffff / 2) return LBM_ERR_ARG;
    if (!(c.tau0 > 0.5) || !std::isfinite(c.tau0)) return LBM_ERR_ARG;
    if (!(c.smag_c >= 0.0) || !std::isfinite(c.smag_c)) return LBM_ERR_ARG;
    if (!(c.rho0 > 0.0) || !std::isfinite(c.rho0)) return LBM_ERR_ARG;
    if (!finite_all(c.body_force, 3)) return LBM_ERR_ARG;
    if (c.storage < 0 || c.storage > 2) return LBM_ERR_ARG;
    if (c.bb_mode < 0 || c.bb_mode > 1) return LBM_ERR_ARG;
    if (c.max_bodies < 0 || c.max_walls < 0 || c.max_walls > kMaxWalls) return LBM_ERR_ARG;
    if ((long long)c.max_bodies + c.max_walls > kMaxIds) return LBM_ERR_ARG;
    if (c.nan_guard_every < 0) return LBM_ERR_ARG;

    lbm_ctx *h = new (std::nothrow) lbm_ctx();
    if (!h) return LBM_ERR_OOM;
    h->cfg = c;
    h->stream = (hipStream_t)c.stream;
    h->static_fix_err = static_fix_scratch(&h->static_fix);  // on the current device, once per device
    h->N = (int)N;
    h->Ns = pop_stride(h->N);
    h->sbytes = c.storage == 0 ? 4 : 2;
    auto bail = [&](lbm_status st) {
        lbm_destroy(h);
        return st;
    };
    const size_t popb = (size_t)kQ * h->Ns * h->sbytes;
    const int nbt = c.max_bodies + c.max_walls;
    // tile shape: 64 nodes along x unless x is a multiple of 32 but not of 64
    set_tile_shape(h, (c.nx % 64 != 0 && (c.nx % 32 == 0 || c.nx < 32)) ? kTile32x4x2 : kTile64x2x2);
    if (dalloc(h, &h->pop[0], popb) != hipSuccess || dalloc(h, &h->pop[1], popb) != hipSuccess ||
        dalloc(h, &h->own, sizeof(uint16_t) * N + 4) != hipSuccess ||
        dalloc(h, &h->wall_map, (size_t)N) != hipSuccess ||
        dalloc(h, &h->tab[0], sizeof(double) * kBodyStride * std::max(c.max_bodies, 1)) != hipSuccess ||
        dalloc(h, &h->tab[1], sizeof(double) * kBodyStride * std::max(c.max_bodies, 1)) != hipSuccess ||
        dalloc(h, &h->walls, sizeof(double) * kWallStride * std::max(c.max_walls, 1)) != hipSuccess ||
        dalloc(h, &h->wrec, sizeof(double) * kBodyStride * std::max(c.max_walls, 1)) != hipSuccess ||
        dalloc(h, &h->acc, sizeof(double) * 6 * std::max(nbt, 1)) != hipSuccess ||
        dalloc(h, &h->fsum[0], sizeof(unsigned long long) * std::max(fsum_entries(c), (size_t)1)) != hipSuccess ||
        dalloc(h, &h->fsum[1], sizeof(unsigned long long) * std::max(fsum_entries(c), (size_t)1)) != hipSuccess ||
        dalloc(h, &h->order, sizeof(int) * std::max(c.max_bodies, 1)) != hipSuccess ||
        dalloc(h, &h->zstate, sizeof(ZiebState)) != hipSuccess ||
        dalloc(h, &h->zpart, sizeof(double) * (3 * kZiebMaxBlocks + 1)) != hipSuccess ||
        dalloc(h, &h->flag, sizeof(int)) != hipSuccess)
        return bail(LBM_ERR_OOM);
    if (cleared(hipHostMalloc((void **)&h->pinned, sizeof(double) * kBodyStride * std::max(c.max_bodies, 1))) !=
            hipSuccess ||
        cleared(hipHostMalloc((void **)&h->forces_pin, sizeof(double) * 6 * std::max(nbt, 1))) != hipSuccess ||
        cleared(hipHostMalloc((void **)&h->order_pin, sizeof(int) * std::max(c.max_bodies, 1))) != hipSuccess ||
        cleared(hipHostMalloc((void **)&h->flag_host, sizeof(int))) != hipSuccess)
        return bail(LBM_ERR_OOM);
    if (hipEventCreateWithFlags(&h->stage_evt, hipEventDisableTiming) != hipSuccess) return bail(LBM_ERR_HIP);
    if (hipMemsetAsync(h->wall_map, 0, (size_t)N, h->stream) != hipSuccess ||
        hipMemsetAsync(h->pop[0], 0, popb, h->stream) != hipSuccess ||
        hipMemsetAsync(h->pop[1], 0, popb, h->stream) != hipSuccess ||
        hipMemsetAsync(h->acc, 0, sizeof(double) * 6 * std::max(nbt, 1), h->stream) != hipSuccess ||
        hipMemsetAsync(h->fsum[0], 0, sizeof(unsigned long long) * std::max(fsum_entries(c), (size_t)1), h->stream) !=
            hipSuccess ||
        hipMemsetAsync(h->fsum[1], 0, sizeof(unsigned long long) * std::max(fsum_entries(c), (size_t)1), h->stream) !=
            hipSuccess ||
        hipMemsetAsync(h->flag, 0, sizeof(int), h->stream) != hipSuccess ||
        hipMemsetAsync(h->zpart + 3 * kZiebMaxBlocks, 0, sizeof(double), h->stream) != hipSuccess)
        return bail(LBM_ERR_HIP);
    if (rasterize_full(h) != LBM_OK) return bail(LBM_ERR_HIP);
    if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(LBM_ERR_HIP);
    *out = h;
    return LBM_OK;
}

void lbm_destroy(lbm_handle h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    free_wall_links(h);
    void *dev[] = {h->pop[0], h->pop[1], h->own, h->wall_map, h->tab[0], h->tab[1], h->walls, h->wrec,
                   h->acc, h->fsum[0], h->fsum[1], h->order, h->flag, h->scratch, h->zstate, h->zpart};
    for (void *p : dev)
        if (p) (void)hipFree(p);
    if (h->pinned) (void)hipHostFree(h->pinned);
    if (h->forces_pin) (void)hipHostFree(h->forces_pin);
    if (h->order_pin) (void)hipHostFree(h->order_pin);
    if (h->flag_host) (void)hipHostFree(h->flag_host);
    if (h->stage_evt) (void)hipEventDestroy(h->stage_evt);
    delete h;
}

lbm_status lbm_set_stream(lbm_handle h, void *stream)
{
    if (!h) return LBM_ERR_ARG;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->stream = (hipStream_t)stream;
    h->cfg.stream = stream;
    return LBM_OK;
}

lbm_status lbm_set_walls(lbm_handle h, const uint8_t *wall_id, int32_t n_walls, const double *wall_vel,
                         const double *wall_ref)
{
    if (!h) return LBM_ERR_ARG;
    if (h->initialized) return fail(h, LBM_ERR_STATE, "walls must be set before lbm_init_fields");
    if (!wall_id) return fail(h, LBM_ERR_ARG, "wall_id is NULL");
    if (n_walls < 0) return fail(h, LBM_ERR_ARG, "n_walls < 0");
    if (n_walls > h->cfg.max_walls) return fail(h, LBM_ERR_CAPACITY, "n_walls %d > max_walls %d", n_walls, h->cfg.max_walls);
    if (n_walls > 0 && !wall_vel) return fail(h, LBM_ERR_ARG, "wall_vel is NULL");
    if (n_walls > 0 && !finite_all(wall_vel, 3 * (size_t)n_walls)) return fail(h, LBM_ERR_ARG, "non-finite wall velocity");
    if (wall_ref && n_walls > 0 && !finite_all(wall_ref, 3 * (size_t)n_walls))
        return fail(h, LBM_ERR_ARG, "non-finite wall reference");
    for (int n = 0; n < h->N; ++n)
        if (wall_id[n] > n_walls) return fail(h, LBM_ERR_ARG, "wall id %d at node %d exceeds n_walls", wall_id[n], n);
    std::vector<double> wt((size_t)kWallStride * std::max(n_walls, 1), 0.0);
    for (int w = 0; w < n_walls; ++w)
        for (int a = 0; a < 3; ++a) {
            wt[w * kWallStride + a] = wall_vel[3 * w + a];
            wt[w * kWallStride + 3 + a] = wall_ref ? wall_ref[3 * w + a] : 0.0;
        }
    TRY(copy_sync(h, h->wall_map, wall_id, (size_t)h->N, hipMemcpyHostToDevice));
    TRY(copy_sync(h, h->walls, wt.data(), sizeof(double) * wt.size(), hipMemcpyHostToDevice));
    TRY(upload_wall_records(h, wt.data(), n_walls));
    h->wall_host.assign(wall_id, wall_id + h->N);
    TRY(build_wall_links(h, wall_id, n_walls));
    h->n_walls = n_walls;
    return rasterize_full(h);
}

// The low 21 bits of v spread to every third bit.
static uint64_t spread3(uint64_t v)
{
    v &= 0x1FFFFF;
    v = (v | v << 32) & 0x1F00000000FFFFull;
    v = (v | v << 16) & 0x1F0000FF0000FFull;
    v = (v | v << 8) & 0x100F00F00F00F00Full;
    v = (v | v << 4) & 0x10C30C30C30C30C3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
}

// Interleaved bits of the centre's cell (8 nodes a side) on each axis.
static uint64_t morton_key(const double *X)
{
    return spread3((uint64_t)(X[0] / 8.0)) | spread3((uint64_t)(X[1] / 8.0)) << 1 |
           spread3((uint64_t)(X[2] / 8.0)) << 2;
}

static lbm_status stage_bodies(lbm_ctx *h, int32_t n)
{
    // the link pass takes the spheres in Morton order of their centres, so
    // that the workgroups on one XCD work on neighbouring spheres, which
    // share population lines.  The order changes no result, and spheres move
    // little between calls: it is made again when the count changes, else
    // every 32nd call.
    HIP_TRY(h, hipMemcpyAsync(h->tab[1 - h->ts], h->pinned, sizeof(double) * kBodyStride * (size_t)n,
                              hipMemcpyHostToDevice, h->stream));
    if (n != h->n_order || ++h->order_age >= 32) {
        std::vector<std::pair<uint64_t, int>> keys((size_t)n);
        for (int b = 0; b < n; ++b) keys[(size_t)b] = {morton_key(h->pinned + (size_t)b * kBodyStride), b};
        std::sort(keys.begin(), keys.end());
        for (int b = 0; b < n; ++b) h->order_pin[b] = keys[(size_t)b].second;
        if (n > 0)
            HIP_TRY(h, hipMemcpyAsync(h->order, h->order_pin, sizeof(int) * (size_t)n, hipMemcpyHostToDevice,
                                      h->stream));
        h->n_order = n;
        h->order_age = 0;
    }
    HIP_TRY(h, hipEventRecord(h->stage_evt, h->stream));
    h->nb_next = n;
    h->dirty = true;
    return LBM_OK;
}

lbm_status lbm_set_bodies(lbm_handle h, int32_t n, const double *X, const double *V, const double *Omega,
                          const double *R)
{
    if (!h) return LBM_ERR_ARG;
    if (n < 0) return fail(h, LBM_ERR_ARG, "n < 0");
    if (n > h->cfg.max_bodies) return fail(h, LBM_ERR_CAPACITY, "n %d > max_bodies %d", n, h->cfg.max_bodies);
    if (n > 0 && (!X || !V || !Omega || !R)) return fail(h, LBM_ERR_ARG, "NULL body array");
    const double dims[3] = {(double)h->cfg.nx, (double)h->cfg.ny, (double)h->cfg.nz};
    const double rmax = 0.5 * std::min(dims[0], std::min(dims[1], dims[2])) - 1.0;
    for (int b = 0; b < n; ++b) {
        for (int a = 0; a < 3; ++a) {
            if (!(X[3 * b + a] >= 0.0 && X[3 * b + a] < dims[a]))
                return fail(h, LBM_ERR_ARG, "sphere %d centre outside [0, n) on axis %d", b, a);
            if (!std::isfinite(V[3 * b + a]) || !std::isfinite(Omega[3 * b + a]))
                return fail(h, LBM_ERR_ARG, "sphere %d has a non-finite velocity", b);
        }
        if (!(R[b] > 0.0 && R[b] < rmax))
            return fail(h, LBM_ERR_ARG, "sphere %d radius %g outside (0, %g)", b, R[b], rmax);
    }
    HIP_TRY(h, hipEventSynchronize(h->stage_evt));  // staging buffer free again
    for (int b = 0; b < n; ++b) {
        double *t = h->pinned + (size_t)b * kBodyStride;
        for (int a = 0; a < 3; ++a) {
            t[a] = X[3 * b + a];
            t[3 + a] = V[3 * b + a];
            t[6 + a] = Omega[3 * b + a];
        }
        t[9] = R[b];
    }
    return stage_bodies(h, n);
}

lbm_status lbm_set_bodies_device(lbm_handle h, int32_t n, const double *d_table)
{
    if (!h) return LBM_ERR_ARG;
    if (n < 0) return fail(h, LBM_ERR_ARG, "n < 0");
    if (n > h->cfg.max_bodies) return fail(h, LBM_ERR_CAPACITY, "n %d > max_bodies %d", n, h->cfg.max_bodies);
    if (n > 0 && !d_table) return fail(h, LBM_ERR_ARG, "d_table is NULL");
    if (n > 0)
        HIP_TRY(h, hipMemcpyAsync(h->tab[1 - h->ts], d_table, sizeof(double) * kBodyStride * (size_t)n,
                                  hipMemcpyDeviceToDevice, h->stream));
    h->nb_next = n;
    h->dirty = true;
    return LBM_OK;
}

lbm_status lbm_init_fields(lbm_handle h, const double *rho, const double *u)
{
    if (!h) return LBM_ERR_ARG;
    const size_t N = (size_t)h->N;
    if (rho)
        for (size_t n = 0; n < N; ++n)
            if (!(rho[n] > 0.0) || !std::isfinite(rho[n])) return fail(h, LBM_ERR_ARG, "rho[%zu] not positive and finite", n);
    if (u && !finite_all(u, 3 * N)) return fail(h, LBM_ERR_ARG, "non-finite initial velocity");
    if (h->dirty) {
        h->ts = 1 - h->ts;
        h->nb_state = h->nb_next;
        h->dirty = false;
    }
    TRY(rasterize_full(h));
    const double *rho_dev = nullptr, *u_dev = nullptr;
    if (rho || u) TRY(ensure_scratch(h));
    if (rho) {
        TRY(copy_sync(h, h->scratch, rho, sizeof(double) * N, hipMemcpyHostToDevice));
        rho_dev = h->scratch;
    }
    if (u) {
        TRY(copy_sync(h, h->scratch + N, u, sizeof(double) * 3 * N, hipMemcpyHostToDevice));
        u_dev = h->scratch + N;
    }
    GeomArgs g = geom(h);
    HIP_TRY(h, launch_init_pop(h->cfg.storage, g, rho_dev, u_dev, h->stream));
    HIP_TRY(h, launch_zero(h->acc, 6 * (h->cfg.max_bodies + h->cfg.max_walls), h->stream));
    TRY(reset_sums(h));
    TRY(clear_flag(h));
    const ZiebState z0{-1.0, 0.0, 0.0, 0.0};
    HIP_TRY(h, hipMemcpyAsync(h->zstate, &z0, sizeof z0, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->initialized = true;
    h->steps_done = 0;
    h->geom_gen++;
    return LBM_OK;
}

}  // extern "C"

namespace {

// One step of the handle: inflow-plane update, re-rasterisation when the
// bodies changed, then the fused step kernel (which also finishes the force
// sums of the step before, if nothing read them), or (the split path) the
// boundary-link pass and the pull-collide kernel.  With fix, the fused kernel
// runs whatever the path, its force sums going to fix (bodies first, then the
// wall copies right after them) instead of the handle's buffers.
lbm_status step_once(lbm_ctx *h, unsigned long long *fix = nullptr)
{
    const lbm_config &c = h->cfg;
    std::array<hipEvent_t, 4> ev{};
    // a profiled step: every prof_every-th while profiling is on (each event
    // costs the step a few microseconds of GPU time)
    const bool prof = h->prof && (h->prof_n++ % h->prof_every) == 0;
    if (prof) HIP_TRY(h, prof_mark(h, &ev[0]));
    // the inflow plane's mean velocity is that of the current state, on its
    // own geometry: taken before the spheres of this step are drawn
    if (h->zieb_z >= 0) HIP_TRY(h, launch_zieb_update(c.storage, zieb_args(h), h->stream));
    if (h->dirty) TRY(rasterize_update(h));
    if (fix || h->path == LBM_PATH_FUSED) {
        // profiled: the fused kernel's own start and end (ev[1], ev[3]),
        // recorded by its launch
        if (prof) {
            HIP_TRY(h, prof_event(h, &ev[1]));
            HIP_TRY(h, prof_event(h, &ev[3]));
        }
        ev[2] = ev[1];
        FusedArgs f = fused_args(h);
        if (fix) {
            f.fsum = fix;
            f.wall_base = h->nb_state;
        }
        if (h->fpending) {  // the last step's forces, unread: into acc by this launch
            f.fin = pending_finish(h);
            h->fpending = false;
        }
        HIP_TRY(h, launch_fused(c.storage, f, h->stream, ev[1], ev[3]));
        h->pend = FinishArgs{f.fsum, f.wall_base, h->nb_state, h->n_walls, h->acc, nullptr};
        h->fpending = true;
        if (!fix) h->fcur ^= 1;
    } else {
        if (prof) HIP_TRY(h, prof_mark(h, &ev[1]));
        TRY(finish_forces(h, nullptr));
        LinkArgs la = link_args(h);
        HIP_TRY(h, launch_links(c.storage, la, h->stream));
        if (prof) HIP_TRY(h, prof_mark(h, &ev[2]));
        // the step kernel's first workgroups add up the wall chunks
        StepArgs a = step_args(h);
        a.n_wsum = la.n_walls;
        a.wsum_nb = la.nb;
        a.wsum_part = h->wl_part;
        a.wsum_wblk = h->wl_wblk;
        a.wsum_out = h->acc;
        HIP_TRY(h, launch_step(c.storage, a, h->stream));
        if (prof) HIP_TRY(h, prof_mark(h, &ev[3]));
    }
    if (prof) h->prof_ev.push_back(ev);
    h->cur = 1 - h->cur;
    h->steps_done++;
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_step(lbm_handle h, int32_t nsteps)
{
    if (!h) return LBM_ERR_ARG;
    if (nsteps < 0) return fail(h, LBM_ERR_ARG, "nsteps < 0");
    lbm_status st = check_ready(h);
    if (st != LBM_OK) return st;
    const lbm_config &c = h->cfg;
    for (int s = 0; s < nsteps; ++s) {
        TRY(step_once(h));
        if (c.nan_guard_every > 0 && (h->steps_done % c.nan_guard_every == 0 || s == nsteps - 1)) {
            HIP_TRY(h, hipMemcpyAsync(h->flag_host, h->flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
            HIP_TRY(h, hipStreamSynchronize(h->stream));
            if (*h->flag_host)
                return fail(h, LBM_ERR_UNSTABLE, "non-finite or non-positive density/velocity by step %d",
                            h->steps_done);
        }
    }
    return LBM_OK;
}

static_assert(kStaticFixHalf == LBM_STATIC_FIX_SUMS && kWallRep == 64, "static force scratch as documented");

lbm_status lbm_step_noalloc(lbm_handle h, int32_t nsteps)
{
    if (!h) return LBM_ERR_ARG;
    if (nsteps < 0) return fail(h, LBM_ERR_ARG, "nsteps < 0");
    lbm_status st = check_ready(h);
    if (st != LBM_OK) return st;
    if (!h->static_fix)
        return fail(h, LBM_ERR_HIP, "static force scratch unavailable: %s", hipGetErrorString(h->static_fix_err));
    const int nb = std::max(h->nb_state, h->dirty ? h->nb_next : 0);
    const size_t need = 6 * ((size_t)nb + (size_t)h->n_walls * kWallRep);
    if (need > (size_t)kStaticFixHalf)
        return fail(h, LBM_ERR_CAPACITY,
                    "%d bodies and %d walls need %zu fixed-point sums per step; the static scratch holds %d",
                    nb, h->n_walls, need, kStaticFixHalf);
    if (nsteps == 0) return LBM_OK;
    const lbm_config &c = h->cfg;
    // the halves start at zero (a previous call may have stopped early);
    // cleared by a kernel, not a memset node, should the call be captured
    HIP_TRY(h, launch_zero_fix(h->static_fix, kStaticFixHalf + (int)need, h->stream));
    const bool prof = h->prof;
    h->prof = false;  // no events: the profile pool may grow
    st = LBM_OK;
    for (int s = 0; s < nsteps && st == LBM_OK; ++s) {
        st = step_once(h, h->static_fix + (size_t)(s & 1) * kStaticFixHalf);
        if (st == LBM_OK && c.nan_guard_every > 0 && (h->steps_done % c.nan_guard_every == 0 || s == nsteps - 1)) {
            hipError_t e = hipMemcpyAsync(h->flag_host, h->flag, sizeof(int), hipMemcpyDeviceToHost, h->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess)
                st = fail(h, LBM_ERR_HIP, "%s", hipGetErrorString(e));
            else if (*h->flag_host)
                st = fail(h, LBM_ERR_UNSTABLE, "non-finite or non-positive density/velocity by step %d", h->steps_done);
        }
    }
    h->prof = prof;
    // nothing may stay pending in the shared array when the call returns
    const lbm_status fst = finish_forces(h, nullptr);
    return st != LBM_OK ? st : fst;
}

lbm_status lbm_get_forces(lbm_handle h, double *F, double *T)
{
    if (!h) return LBM_ERR_ARG;
    lbm_status st = check_ready(h);
    if (st != LBM_OK) return st;
    const int nbt = h->nb_state + h->n_walls;
    if (nbt > 0 && (!F || !T)) return fail(h, LBM_ERR_ARG, "NULL output");
    TRY(finish_forces(h, nullptr));
    // through the pinned staging buffer: one DMA, no per-call allocation
    const double *buf = h->forces_pin;
    HIP_TRY(h, hipMemcpyAsync(h->forces_pin, h->acc, sizeof(double) * 6 * nbt, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    for (int b = 0; b < nbt; ++b)
        for (int a = 0; a < 3; ++a) {
            F[3 * b + a] = buf[6 * b + a];
            T[3 * b + a] = buf[6 * b + 3 + a];
        }
    return LBM_OK;
}

lbm_status lbm_get_forces_device(lbm_handle h, double *d_out)
{
    if (!h) return LBM_ERR_ARG;
    lbm_status st = check_ready(h);
    if (st != LBM_OK) return st;
    const int nbt = h->nb_state + h->n_walls;
    if (nbt > 0 && !d_out) return fail(h, LBM_ERR_ARG, "NULL output");
    if (h->fpending) return finish_forces(h, d_out);  // one launch: acc and the caller's copy
    if (nbt > 0)
        HIP_TRY(h, hipMemcpyAsync(d_out, h->acc, sizeof(double) * 6 * nbt, hipMemcpyDeviceToDevice, h->stream));
    return LBM_OK;
}

lbm_status lbm_get_populations(lbm_handle h, double *f)
{
    if (!h || !f) return h ? fail(h, LBM_ERR_ARG, "NULL output") : LBM_ERR_ARG;
    lbm_status st = check_ready(h);
    if (st != LBM_OK) return st;
    if ((st = ensure_scratch(h)) != LBM_OK) return st;
    GeomArgs g = geom(h);
    for (int i = 0; i < kQ; ++i) {
        HIP_TRY(h, launch_export_pop(h->cfg.storage, g, h->walls, i, h->scratch, h->stream));
        HIP_TRY(h, hipMemcpyAsync(f + (size_t)i * h->N, h->scratch, sizeof(double) * h->N, hipMemcpyDeviceToHost,
                                  h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    return LBM_OK;
}

lbm_status lbm_set_populations(lbm_handle h, const double *f)
{
    if (!h || !f) return h ? fail(h, LBM_ERR_ARG, "NULL input") : LBM_ERR_ARG;
    lbm_status st = check_ready(h);
    if (st != LBM_OK) return st;
    if (!finite_all(f, (size_t)kQ * h->N)) return fail(h, LBM_ERR_ARG, "non-finite populations");
    if ((st = ensure_scratch(h)) != LBM_OK) return st;
    for (int i = 0; i < kQ; ++i) {
        TRY(copy_sync(h, h->scratch, f + (size_t)i * h->N, sizeof(double) * h->N, hipMemcpyHostToDevice));
        HIP_TRY(h, launch_import_pop(h->cfg.storage, h->N, h->Ns, i, (float)h->cfg.rho0, h->scratch, h->pop[h->cur],
                                     h->stream));
    }
    TRY(clear_flag(h));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

lbm_status lbm_get_macro(lbm_handle h, double *rho, double *u)
{
    if (!h || !rho || !u) return h ? fail(h, LBM_ERR_ARG, "NULL output") : LBM_ERR_ARG;
    TRY(check_ready(h));
    TRY(ensure_scratch(h));
    const size_t N = (size_t)h->N;
    GeomArgs g = geom(h);
    HIP_TRY(h, launch_export_macro(h->cfg.storage, g, h->walls, h->cfg.body_force[0], h->cfg.body_force[1],
                                   h->cfg.body_force[2], h->scratch, h->scratch + N, h->stream));
    TRY(copy_sync(h, rho, h->scratch, sizeof(double) * N, hipMemcpyDeviceToHost));
    TRY(copy_sync(h, u, h->scratch + N, sizeof(double) * 3 * N, hipMemcpyDeviceToHost));
    return LBM_OK;
}

lbm_status lbm_get_owner(lbm_handle h, int32_t *owner)
{
    if (!h || !owner) return h ? fail(h, LBM_ERR_ARG, "NULL output") : LBM_ERR_ARG;
    lbm_status st = ensure_scratch(h);
    if (st != LBM_OK) return st;
    int32_t *d = reinterpret_cast<int32_t *>(h->scratch);
    HIP_TRY(h, launch_export_owner(h->own, h->N, d, h->stream));
    HIP_TRY(h, hipMemcpyAsync(owner, d, sizeof(int32_t) * h->N, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

namespace {
struct StateHeader {
    char magic[8];
    int32_t version, nx, ny, nz, storage, n_walls, nb_state, nb_next, dirty, steps_done, max_bodies, max_walls;
};
}  // namespace

lbm_status lbm_get_state(lbm_handle h, void *buf, size_t *bytes)
{
    if (!h || !bytes) return h ? fail(h, LBM_ERR_ARG, "NULL size") : LBM_ERR_ARG;
    lbm_status st = check_ready(h);
    if (st != LBM_OK) return st;
    const size_t popb = (size_t)kQ * h->Ns * h->sbytes;
    const size_t tabb = sizeof(double) * kBodyStride * std::max(h->cfg.max_bodies, 1);
    const size_t wallb = sizeof(double) * kWallStride * std::max(h->cfg.max_walls, 1);
    const size_t accb = sizeof(double) * 6 * std::max(h->cfg.max_bodies + h->cfg.max_walls, 1);
    const size_t need = sizeof(StateHeader) + popb + sizeof(uint16_t) * h->N + (size_t)h->N + 2 * tabb + wallb + accb +
                        sizeof(ZiebState);
    if (!buf) {
        *bytes = need;
        return LBM_OK;
    }
    if (*bytes < need) return fail(h, LBM_ERR_ARG, "buffer of %zu bytes < %zu needed", *bytes, need);
    TRY(finish_forces(h, nullptr));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    StateHeader hd{};
    memcpy(hd.magic, "LBMSTAT1", 8);
    hd.version = lbm_version();
    hd.nx = h->cfg.nx;
    hd.ny = h->cfg.ny;
    hd.nz = h->cfg.nz;
    hd.storage = h->cfg.storage;
    hd.n_walls = h->n_walls;
    hd.nb_state = h->nb_state;
    hd.nb_next = h->nb_next;
    hd.dirty = h->dirty;
    hd.steps_done = h->steps_done;
    hd.max_bodies = h->cfg.max_bodies;
    hd.max_walls = h->cfg.max_walls;
    char *p = static_cast<char *>(buf);
    memcpy(p, &hd, sizeof hd);
    p += sizeof hd;
    TRY(copy_sync(h, p, h->pop[h->cur], popb, hipMemcpyDeviceToHost));
    p += popb;
    TRY(copy_sync(h, p, h->own, sizeof(uint16_t) * h->N, hipMemcpyDeviceToHost));
    p += sizeof(uint16_t) * h->N;
    TRY(copy_sync(h, p, h->wall_map, (size_t)h->N, hipMemcpyDeviceToHost));
    p += h->N;
    TRY(copy_sync(h, p, h->tab[h->ts], tabb, hipMemcpyDeviceToHost));
    p += tabb;
    TRY(copy_sync(h, p, h->tab[1 - h->ts], tabb, hipMemcpyDeviceToHost));
    p += tabb;
    TRY(copy_sync(h, p, h->walls, wallb, hipMemcpyDeviceToHost));
    p += wallb;
    TRY(copy_sync(h, p, h->acc, accb, hipMemcpyDeviceToHost));
    p += accb;
    TRY(copy_sync(h, p, h->zstate, sizeof(ZiebState), hipMemcpyDeviceToHost));
    *bytes = need;
    return LBM_OK;
}

lbm_status lbm_set_state(lbm_handle h, const void *buf, size_t bytes)
{
    if (!h || !buf) return h ? fail(h, LBM_ERR_ARG, "NULL buffer") : LBM_ERR_ARG;
    const size_t popb = (size_t)kQ * h->Ns * h->sbytes;
    const size_t tabb = sizeof(double) * kBodyStride * std::max(h->cfg.max_bodies, 1);
    const size_t wallb = sizeof(double) * kWallStride * std::max(h->cfg.max_walls, 1);
    const size_t accb = sizeof(double) * 6 * std::max(h->cfg.max_bodies + h->cfg.max_walls, 1);
    const size_t need = sizeof(StateHeader) + popb + sizeof(uint16_t) * h->N + (size_t)h->N + 2 * tabb + wallb + accb +
                        sizeof(ZiebState);
    if (bytes < need) return fail(h, LBM_ERR_ARG, "state of %zu bytes < %zu expected", bytes, need);
    StateHeader hd;
    memcpy(&hd, buf, sizeof hd);
    if (memcmp(hd.magic, "LBMSTAT1", 8) != 0 || hd.nx != h->cfg.nx || hd.ny != h->cfg.ny || hd.nz != h->cfg.nz ||
        hd.storage != h->cfg.storage || hd.max_bodies != h->cfg.max_bodies || hd.max_walls != h->cfg.max_walls)
        return fail(h, LBM_ERR_ARG, "state does not match this handle's configuration");
    if (hd.nb_state < 0 || hd.nb_state > h->cfg.max_bodies || hd.nb_next < 0 || hd.nb_next > h->cfg.max_bodies ||
        hd.n_walls < 0 || hd.n_walls > h->cfg.max_walls || (hd.dirty != 0 && hd.dirty != 1) || hd.steps_done < 0)
        return fail(h, LBM_ERR_ARG, "state header out of range (bodies %d/%d, walls %d, dirty %d, steps %d)",
                    hd.nb_state, hd.nb_next, hd.n_walls, hd.dirty, hd.steps_done);
    {
        // wall ids of the voxel map within the state's wall count
        const uint8_t *wm = reinterpret_cast<const uint8_t *>(buf) + sizeof hd + popb + sizeof(uint16_t) * h->N;
        for (int n = 0; n < h->N; ++n)
            if (wm[n] > hd.n_walls) return fail(h, LBM_ERR_ARG, "state wall map names wall %d of %d", wm[n], hd.n_walls);
        // owner codes: fluid, or a wall or sphere of the state (the kernels
        // look solid owners up in the wall and body tables)
        const char *op = reinterpret_cast<const char *>(buf) + sizeof hd + popb;
        const int nsolid = hd.n_walls + hd.nb_state;
        for (int n = 0; n < h->N; ++n) {
            uint16_t o;
            memcpy(&o, op + sizeof(uint16_t) * (size_t)n, sizeof o);
            if (o != kFluid && o >= nsolid)
                return fail(h, LBM_ERR_ARG, "state owner map names solid %d at node %d (walls + spheres = %d)", o, n,
                            nsolid);
        }
    }
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    const char *p = static_cast<const char *>(buf) + sizeof hd;
    TRY(copy_sync(h, h->pop[h->cur], p, popb, hipMemcpyHostToDevice));
    p += popb;
    TRY(copy_sync(h, h->own, p, sizeof(uint16_t) * h->N, hipMemcpyHostToDevice));
    p += sizeof(uint16_t) * h->N;
    TRY(copy_sync(h, h->wall_map, p, (size_t)h->N, hipMemcpyHostToDevice));
    h->wall_host.assign(reinterpret_cast<const uint8_t *>(p), reinterpret_cast<const uint8_t *>(p) + h->N);
    TRY(build_wall_links(h, reinterpret_cast<const uint8_t *>(p), hd.n_walls));
    p += h->N;
    TRY(copy_sync(h, h->tab[h->ts], p, tabb, hipMemcpyHostToDevice));
    p += tabb;
    TRY(copy_sync(h, h->tab[1 - h->ts], p, tabb, hipMemcpyHostToDevice));
    p += tabb;
    TRY(copy_sync(h, h->walls, p, wallb, hipMemcpyHostToDevice));
    TRY(upload_wall_records(h, reinterpret_cast<const double *>(p), hd.n_walls));
    p += wallb;
    TRY(copy_sync(h, h->acc, p, accb, hipMemcpyHostToDevice));
    p += accb;
    TRY(copy_sync(h, h->zstate, p, sizeof(ZiebState), hipMemcpyHostToDevice));
    h->n_walls = hd.n_walls;
    h->nb_state = hd.nb_state;
    h->nb_next = hd.nb_next;
    h->dirty = hd.dirty != 0;
    h->steps_done = hd.steps_done;
    h->initialized = true;
    h->geom_gen++;
    TRY(reset_sums(h));
    TRY(clear_flag(h));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

lbm_status lbm_get_info(lbm_handle h, lbm_info *info)
{
    if (!h || !info) return h ? fail(h, LBM_ERR_ARG, "NULL output") : LBM_ERR_ARG;
    info->n_nodes = h->N;
    info->n_bodies = h->nb_state;
    info->n_walls = h->n_walls;
    info->storage_bytes = h->sbytes;
    info->steps_done = h->steps_done;
    info->device_bytes = h->device_bytes;
    return LBM_OK;
}

lbm_status lbm_count_fluid(lbm_handle h, int64_t *n_fluid)
{
    if (!h || !n_fluid) return h ? fail(h, LBM_ERR_ARG, "NULL output") : LBM_ERR_ARG;
    TRY(ensure_scratch(h));
    unsigned long long *d = reinterpret_cast<unsigned long long *>(h->scratch);
    unsigned long long cnt = 0;
    HIP_TRY(h, launch_zero(reinterpret_cast<double *>(d), 1, h->stream));
    HIP_TRY(h, launch_count_fluid(h->own, h->N, d, h->stream));
    TRY(copy_sync(h, &cnt, d, sizeof cnt, hipMemcpyDeviceToHost));
    *n_fluid = (int64_t)cnt;
    return LBM_OK;
}

lbm_status lbm_profile(lbm_handle h, int32_t every)
{
    if (!h) return LBM_ERR_ARG;
    if (every < 0) return fail(h, LBM_ERR_ARG, "profile interval %d < 0", every);
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->prof_ev.clear();
    h->ev_used = 0;
    h->prof = every != 0;
    h->prof_every = every > 0 ? every : 1;
    h->prof_n = 0;
    return LBM_OK;
}

lbm_status lbm_profile_read(lbm_handle h, double *ms_total, int64_t *launches)
{
    if (!h || !ms_total || !launches) return h ? fail(h, LBM_ERR_ARG, "NULL output") : LBM_ERR_ARG;
    double parts[LBM_PROF_PARTS];
    int64_t steps = 0;
    TRY(lbm_profile_read_parts(h, parts, &steps));
    *ms_total = parts[LBM_PROF_STEP];
    *launches = steps;
    return LBM_OK;
}

lbm_status lbm_profile_read_parts(lbm_handle h, double *ms, int64_t *steps)
{
    if (!h || !ms || !steps) return h ? fail(h, LBM_ERR_ARG, "NULL output") : LBM_ERR_ARG;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    double tot[LBM_PROF_PARTS] = {0.0};
    for (const auto &e : h->prof_ev) {
        // parts: geometry, link pass, step kernel, then the whole step
        const int from[LBM_PROF_PARTS] = {0, 1, 2, 0}, to[LBM_PROF_PARTS] = {1, 2, 3, 3};
        for (int p = 0; p < LBM_PROF_PARTS; ++p) {
            if (e[from[p]] == e[to[p]]) continue;
            float v = 0.f;
            HIP_TRY(h, hipEventElapsedTime(&v, e[from[p]], e[to[p]]));
            tot[p] += v;
        }
    }
    for (int p = 0; p < LBM_PROF_PARTS; ++p) ms[p] = tot[p];
    *steps = (int64_t)h->prof_ev.size();
    return LBM_OK;
}

lbm_status lbm_set_step_path(lbm_handle h, int32_t path)
{
    if (!h) return LBM_ERR_ARG;
    if (path != LBM_PATH_FUSED && path != LBM_PATH_SPLIT) return fail(h, LBM_ERR_ARG, "unknown step path %d", path);
    h->path = path;
    return LBM_OK;
}

lbm_status lbm_get_step_path(lbm_handle h, int32_t *path)
{
    if (!h || !path) return h ? fail(h, LBM_ERR_ARG, "NULL output") : LBM_ERR_ARG;
    *path = h->path;
    return LBM_OK;
}

lbm_status lbm_set_zieb(lbm_handle h, int32_t z_s, double area, double volume, double v_piston)
{
    if (!h) return LBM_ERR_ARG;
    if (h->initialized) return fail(h, LBM_ERR_STATE, "the inflow plane must be set before lbm_init_fields");
    const int nx = h->cfg.nx, ny = h->cfg.ny, nz = h->cfg.nz;
    if (z_s < 0) {  // remove the plane
        h->zieb_z = -1;
        if (h->n_walls > 0 && !h->wall_host.empty()) return build_wall_links(h, h->wall_host.data(), h->n_walls);
        return LBM_OK;
    }
    if (z_s >= nz) return fail(h, LBM_ERR_ARG, "z_s %d outside [0, %d)", z_s, nz);
    if (!(area > 0.0) || !(volume > 0.0) || !std::isfinite(area) || !std::isfinite(volume) || !std::isfinite(v_piston))
        return fail(h, LBM_ERR_ARG, "area and volume must be positive and finite, v_piston finite");
    const int zv = (z_s + nz - 1) % nz;
    if (h->wall_host.empty()) return fail(h, LBM_ERR_STATE, "set the walls first: layer z = %d must be wall", zv);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            if (!h->wall_host[(size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * zv)])
                return fail(h, LBM_ERR_ARG, "node (%d, %d, %d) below the inflow plane is not a wall", x, y, zv);
    h->zieb_z = z_s;
    h->zieb_area = area;
    h->zieb_volume = volume;
    h->zieb_vp = v_piston;
    return build_wall_links(h, h->wall_host.data(), h->n_walls);
}

lbm_status lbm_get_zieb(lbm_handle h, double *state)
{
    if (!h || !state) return h ? fail(h, LBM_ERR_ARG, "NULL output") : LBM_ERR_ARG;
    if (h->zieb_z < 0) return fail(h, LBM_ERR_STATE, "no inflow plane");
    ZiebState z{};
    TRY(copy_sync(h, &z, h->zstate, sizeof z, hipMemcpyDeviceToHost));
    state[0] = z.rho;
    state[1] = z.H;
    state[2] = z.vf;
    return LBM_OK;
}

lbm_status lbm_set_body_force(lbm_handle h, const double *F)
{
    if (!h || !F) return h ? fail(h, LBM_ERR_ARG, "NULL force") : LBM_ERR_ARG;
    if (!finite_all(F, 3)) return fail(h, LBM_ERR_ARG, "non-finite body force");
    for (int a = 0; a < 3; ++a) h->cfg.body_force[a] = F[a];
    h->geom_gen++;
    return LBM_OK;
}

lbm_status lbm_drag_gradient(lbm_handle h, int32_t nsteps, int32_t ckpt, double *J, double *dJdF, double *dJdV)
{
    if (!h) return LBM_ERR_ARG;
    TRY(check_ready(h));
    if (nsteps < 1 || ckpt < 1) return fail(h, LBM_ERR_ARG, "nsteps and ckpt must be at least 1");
    if (!J || !dJdF || (h->nb_next > 0 && !dJdV)) return fail(h, LBM_ERR_ARG, "NULL output");
    if (h->cfg.storage != 0) return fail(h, LBM_ERR_ARG, "the drag gradient needs FP32 storage");
    if (h->n_walls > 0) return fail(h, LBM_ERR_ARG, "the drag gradient has no wall links");
    if (h->zieb_z >= 0) return fail(h, LBM_ERR_ARG, "the drag gradient has no inflow plane");
    if (h->dirty) TRY(rasterize_update(h));
    const int nb = h->nb_state;
    const size_t popb = sizeof(float) * kQ * (size_t)h->Ns;
    const int nck = (nsteps + ckpt - 1) / ckpt;
    const int nseg = std::min(ckpt, nsteps);
    // device buffers of this call
    std::vector<void *> bufs;
    bool oom = false;
    auto get = [&](size_t bytes) -> void * {
        void *p = nullptr;
        if (cleared(hipMalloc(&p, bytes ? bytes : 16)) != hipSuccess) {
            oom = true;
            return nullptr;
        }
        bufs.push_back(p);
        return p;
    };
    auto release = [&]() {
        (void)hipStreamSynchronize(h->stream);
        for (void *p : bufs) (void)hipFree(p);
        bufs.clear();
    };
    // every return (an error of a HIP call included) frees the buffers and
    // leaves profiling as it was
    const bool prof = h->prof;
    struct Exit {
        decltype(release) &free_all;
        lbm_ctx *h;
        bool prof;
        ~Exit()
        {
            free_all();
            h->prof = prof;
        }
    } on_exit{release, h, prof};
    std::vector<float *> ck((size_t)nck), seg((size_t)nseg);
    for (auto &b : ck) b = static_cast<float *>(get(popb));
    for (auto &b : seg) b = static_cast<float *>(get(popb));
    float *lam[2] = {static_cast<float *>(get(popb)), static_cast<float *>(get(popb))};
    const int nbt = std::max(nb + h->n_walls, 1);
    double *fscratch = static_cast<double *>(get(sizeof(double) * 6 * (size_t)nbt));
    double *accsave = static_cast<double *>(get(sizeof(double) * 6 * (size_t)nbt));
    double *dF_tile = static_cast<double *>(get(sizeof(double) * 3 * (size_t)h->n_tiles));
    double *dF = static_cast<double *>(get(sizeof(double) * 3));
    double *dV = static_cast<double *>(get(sizeof(double) * 3 * (size_t)std::max(nb, 1)));
    if (oom) return fail(h, LBM_ERR_OOM, "no device memory for %d checkpoints and %d recomputed states", nck, nseg);
    const lbm_config &c = h->cfg;
    // forward, keeping every ckpt-th state: the steps of lbm_step, so that the
    // state and forces left behind are those of plain stepping
    h->prof = false;
    for (int n = 0; n < nsteps; ++n) {
        if (n % ckpt == 0) HIP_TRY(h, hipMemcpyAsync(ck[(size_t)(n / ckpt)], h->pop[h->cur], popb, hipMemcpyDeviceToDevice, h->stream));
        const lbm_status sst = step_once(h);
        if (sst != LBM_OK) return sst;
    }
    h->prof = prof;
    TRY(finish_forces(h, nullptr));
    std::vector<double> acc_h((size_t)6 * nbt);
    TRY(copy_sync(h, acc_h.data(), h->acc, sizeof(double) * 6 * nbt, hipMemcpyDeviceToHost));
    double Jv = 0.0;
    for (int b = 0; b < nb; ++b) Jv += acc_h[(size_t)6 * b];
    HIP_TRY(h, hipMemcpyAsync(accsave, h->acc, sizeof(double) * 6 * nbt, hipMemcpyDeviceToDevice, h->stream));
    // backward: the objective's derivative gives the adjoint of P_{N-1}
    HIP_TRY(h, hipMemsetAsync(dF_tile, 0, sizeof(double) * 3 * h->n_tiles, h->stream));
    HIP_TRY(h, hipMemsetAsync(dV, 0, sizeof(double) * 3 * std::max(nb, 1), h->stream));
    HIP_TRY(h, hipMemsetAsync(lam[0], 0, popb, h->stream));
    LinkArgs lg = link_args(h);
    lg.out = fscratch;
    AdjLinkArgs al{lg, nullptr, lam[0], dV};
    HIP_TRY(h, launch_adj_links(al, h->stream));
    int li = 0;  // lam[li] is the adjoint of P_m
    for (int s = nck - 1; s >= 0; --s) {
        const int start = s * ckpt, end = std::min(start + ckpt, nsteps);
        // recompute P_start .. P_{end-1} of the segment
        HIP_TRY(h, hipMemcpyAsync(seg[0], ck[(size_t)s], popb, hipMemcpyDeviceToDevice, h->stream));
        for (int k = start + 1; k < end; ++k) {
            LinkArgs la = link_args(h);
            la.pop = seg[(size_t)(k - 1 - start)];
            la.out = fscratch;
            HIP_TRY(h, launch_links(c.storage, la, h->stream));
            StepArgs a = step_args(h);
            a.flag = nullptr;
            a.src = seg[(size_t)(k - 1 - start)];
            a.dst = seg[(size_t)(k - start)];
            HIP_TRY(h, launch_step(c.storage, a, h->stream));
        }
        // steps m = k + 1 whose source P_k lies in the segment, m from N - 1 down
        for (int m = std::min(end, nsteps - 1); m >= start + 1; --m) {
            float *src = seg[(size_t)(m - 1 - start)];
            if (m == end) {
                // the recompute stopped before step end: put its link values
                // into the solid slots of P_{end-1}; for earlier steps the
                // recompute's own link pass left them there
                LinkArgs la = link_args(h);
                la.pop = src;
                la.out = fscratch;
                HIP_TRY(h, launch_links(c.storage, la, h->stream));
            }
            StepArgs a = step_args(h);
            a.flag = nullptr;
            a.src = src;
            AdjStepArgs ga{a, lam[li], lam[1 - li], dF_tile};
            HIP_TRY(h, launch_adj_collide(ga, h->stream));
            AdjLinkArgs am{lg, lam[1 - li], lam[1 - li], dV};
            HIP_TRY(h, launch_adj_links(am, h->stream));
            li = 1 - li;
        }
    }
    HIP_TRY(h, launch_adj_reduce(dF_tile, h->n_tiles, dF, h->stream));
    HIP_TRY(h, hipMemcpyAsync(h->acc, accsave, sizeof(double) * 6 * nbt, hipMemcpyDeviceToDevice, h->stream));
    TRY(copy_sync(h, dJdF, dF, sizeof(double) * 3, hipMemcpyDeviceToHost));
    if (nb > 0) TRY(copy_sync(h, dJdV, dV, sizeof(double) * 3 * nb, hipMemcpyDeviceToHost));
    *J = Jv;
    return LBM_OK;
}

lbm_status lbm_set_tile(lbm_handle h, int32_t shape)
{
    if (!h) return LBM_ERR_ARG;
    if (shape < 0 || shape >= kNumTileShapes)
        return fail(h, LBM_ERR_ARG, "tile shape %d not in [0, %d)", shape, kNumTileShapes);
    set_tile_shape(h, shape);
    return LBM_OK;
}

lbm_status lbm_get_tile(lbm_handle h, int32_t *shape)
{
    if (!h || !shape) return h ? fail(h, LBM_ERR_ARG, "NULL output") : LBM_ERR_ARG;
    *shape = h->tile;
    return LBM_OK;
}

lbm_status lbm_autotune_tile(lbm_handle h, int32_t trial_steps, const char *cache_path, int32_t *shape_out,
                             double *us)
{
    if (!h) return LBM_ERR_ARG;
    TRY(check_ready(h));
    if (trial_steps < 1) return fail(h, LBM_ERR_ARG, "trial_steps < 1");
    if (h->dirty) return fail(h, LBM_ERR_STATE, "bodies were set since the last step; step before tuning");
    if (us)
        for (int k = 0; k < kNumTileShapes; ++k) us[k] = -1.0;
    static const char *kStorage[] = {"f32", "f16", "bf16"};
    const std::string key = arch_name() + "/" + kStorage[h->cfg.storage] + "/" + std::to_string(h->cfg.nx) + "x" +
                            std::to_string(h->cfg.ny) + "x" + std::to_string(h->cfg.nz);
    std::map<std::string, int> cache;
    if (cache_path) {
        cache = read_cache(cache_path);
        auto it = cache.find(key);
        if (it != cache.end() && it->second >= 0 && it->second < kNumTileShapes) {
            set_tile_shape(h, it->second);
            if (shape_out) *shape_out = it->second;
            return LBM_OK;
        }
    }
    // The step kernel reads the current state and writes only the spare
    // buffer (and, on the fused path, the force sums, cleared afterwards), so
    // repeated launches leave the state as it is.
    // Two passes over the shapes, each shape's best pass kept: a GPU that
    // has just started stepping runs the first trials slow (by up to a tenth
    // on the duct), which one pass would charge to the shapes timed first.
    EventPair ev;
    HIP_TRY(h, ev.create());
    const bool fused = h->path == LBM_PATH_FUSED;
    double t_best[kNumTileShapes];
    for (int pass = 0; pass < 2; ++pass)
        for (int k = 0; k < kNumTileShapes; ++k) {
            set_tile_shape(h, k);
            FusedArgs f = fused_args(h);
            f.s.flag = nullptr;
            auto launch = [&]() {
                return fused ? launch_fused(h->cfg.storage, f, h->stream)
                             : launch_step(h->cfg.storage, f.s, h->stream);
            };
            HIP_TRY(h, launch());
            HIP_TRY(h, hipEventRecord(ev.e0, h->stream));
            for (int i = 0; i < trial_steps; ++i) HIP_TRY(h, launch());
            HIP_TRY(h, hipEventRecord(ev.e1, h->stream));
            HIP_TRY(h, hipEventSynchronize(ev.e1));
            float ms = 0.f;
            HIP_TRY(h, hipEventElapsedTime(&ms, ev.e0, ev.e1));
            const double t = 1e3 * ms / trial_steps;
            t_best[k] = pass == 0 ? t : std::min(t_best[k], t);
        }
    int best = 0;
    for (int k = 0; k < kNumTileShapes; ++k) {
        if (us) us[k] = t_best[k];
        if (t_best[k] < t_best[best]) best = k;
    }
    set_tile_shape(h, best);
    HIP_TRY(h, launch_zero_fix(h->fsum[h->fcur], (int)fsum_entries(h->cfg), h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (shape_out) *shape_out = best;
    if (cache_path) {
        cache[key] = best;
        if (!write_cache(cache_path, cache)) return fail(h, LBM_ERR_ARG, "cannot write %s", cache_path);
    }
    return LBM_OK;
}

}  // extern "C"

struct lbm_batch_ctx {
    std::vector<lbm_ctx *> m;
    std::vector<uint64_t> gen;     // members' geometry generations when the batch was built
    int storage = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    BatchMember *d_members = nullptr;
    int *d_cur = nullptr;
    int *d_queue = nullptr;        // kQueueInts: tile queues, zero between steps
    int *h_cur = nullptr;          // pinned
    BatchStepArgs bs{};
    int shape = kTile64x2x2;       // tile shape of the batched step kernel
    int grid_step = 0;
    // captured graphs: one step, and a block of kBatchBlock steps
    hipGraph_t graph1 = nullptr, graphB = nullptr;
    hipGraphExec_t exec1 = nullptr, execB = nullptr;
    std::string err;
};

namespace {

constexpr int kBatchBlock = 50;    // steps per replay of the block graph

lbm_status bfail(lbm_batch_ctx *b, lbm_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b) b->err = buf;
    return st;
}

#define BHIP_TRY(b, expr)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return bfail((b), e_ == hipErrorOutOfMemory ? LBM_ERR_OOM : LBM_ERR_HIP, "%s: %s", #expr, \
                         hipGetErrorString(e_));                                                 \
    } while (0)

// Queue one batched step: the fused step of every member as one persistent
// launch over their tiles, the forces of every member, and the parity flip.
lbm_status batch_enqueue(lbm_batch_ctx *b)
{
    BHIP_TRY(b, launch_batch_step(b->storage, b->shape, b->bs, b->grid_step, b->stream));
    BHIP_TRY(b, launch_batch_finish(b->bs, b->stream));
    BHIP_TRY(b, launch_batch_flip(b->d_cur, (int)b->m.size(), b->d_queue, b->stream));
    return LBM_OK;
}

void batch_release(lbm_batch_ctx *b)
{
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (hipGraphExec_t *e : {&b->exec1, &b->execB})
        if (*e) {
            (void)hipGraphExecDestroy(*e);
            *e = nullptr;
        }
    for (hipGraph_t *g : {&b->graph1, &b->graphB})
        if (*g) {
            (void)hipGraphDestroy(*g);
            *g = nullptr;
        }
    if (b->d_members) (void)hipFree(b->d_members);
    b->d_members = nullptr;
}

// Capture `steps` batched steps into a graph and instantiate it.
lbm_status batch_capture(lbm_batch_ctx *b, int steps, hipGraph_t *graph, hipGraphExec_t *exec)
{
    BHIP_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    lbm_status st = LBM_OK;
    for (int k = 0; k < steps && st == LBM_OK; ++k) st = batch_enqueue(b);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->stream, &g);
    if (st != LBM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    BHIP_TRY(b, ec);
    *graph = g;
    BHIP_TRY(b, hipGraphInstantiate(exec, g, nullptr, nullptr, 0));
    return LBM_OK;
}

// Member tables for the batch's tile shape, the step kernel's persistent
// grid size, and the captured graphs.
lbm_status batch_build(lbm_batch_ctx *b)
{
    batch_release(b);
    const int n = (int)b->m.size();
    const int TX = kTileDims[b->shape][0], TY = kTileDims[b->shape][1], TZ = kTileDims[b->shape][2];
    std::vector<BatchMember> hm((size_t)n);
    b->gen.assign((size_t)n, 0);
    int tiles = 0, forces = 0;
    for (int i = 0; i < n; ++i) {
        lbm_ctx *h = b->m[(size_t)i];
        BatchMember &bm = hm[(size_t)i];
        bm.f = fused_args(h);
        bm.f.fin = FinishArgs{};
        StepArgs &st = bm.f.s;
        st.flag = nullptr;
        st.tile = b->shape;
        st.ntx = (h->cfg.nx + TX - 1) / TX;
        st.nty = (h->cfg.ny + TY - 1) / TY;
        st.ntz = (h->cfg.nz + TZ - 1) / TZ;
        st.n_tiles = st.ntx * st.nty * st.ntz;
        bm.fin = FinishArgs{h->fsum[h->fcur], h->cfg.max_bodies, h->nb_state, h->n_walls, h->acc, nullptr};
        bm.pop[0] = h->pop[0];
        bm.pop[1] = h->pop[1];
        bm.tile_begin = tiles;
        bm.force_begin = forces;
        tiles += st.n_tiles;
        forces += 6 * (h->nb_state + h->n_walls);
        b->gen[(size_t)i] = h->geom_gen;
    }
    BHIP_TRY(b, cleared(hipMalloc((void **)&b->d_members, sizeof(BatchMember) * (size_t)n)));
    if (!b->d_cur) BHIP_TRY(b, cleared(hipMalloc((void **)&b->d_cur, sizeof(int) * (size_t)n)));
    if (!b->d_queue) {
        BHIP_TRY(b, cleared(hipMalloc((void **)&b->d_queue, sizeof(int) * kQueueInts)));
        BHIP_TRY(b, hipMemsetAsync(b->d_queue, 0, sizeof(int) * kQueueInts, b->stream));
    }
    if (!b->h_cur) BHIP_TRY(b, cleared(hipHostMalloc((void **)&b->h_cur, sizeof(int) * (size_t)n)));
    BHIP_TRY(b, hipMemcpyAsync(b->d_members, hm.data(), sizeof(BatchMember) * (size_t)n, hipMemcpyHostToDevice,
                               b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    b->bs = BatchStepArgs{b->d_members, b->d_cur, b->d_queue, n, tiles, forces};
    int dev = 0, cus = 0;
    BHIP_TRY(b, hipGetDevice(&dev));
    BHIP_TRY(b, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // the persistent step kernel: as many workgroups as are resident at once,
    // a whole number per XCD
    const int rs = batch_step_blocks_per_cu(b->storage, b->shape);
    b->grid_step = std::max(8, std::min(cus * rs / 8 * 8, (tiles + 7) / 8 * 8));
    lbm_status st = batch_capture(b, 1, &b->graph1, &b->exec1);
    if (st == LBM_OK) st = batch_capture(b, kBatchBlock, &b->graphB, &b->execB);
    return st;
}

}  // namespace

extern "C" {

void lbm_batch_destroy(lbm_batch b)
{
    if (!b) return;
    batch_release(b);
    if (b->d_cur) (void)hipFree(b->d_cur);
    if (b->d_queue) (void)hipFree(b->d_queue);
    if (b->h_cur) (void)hipHostFree(b->h_cur);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

const char *lbm_batch_last_error(lbm_batch b) { return b ? b->err.c_str() : "null lbm_batch"; }

lbm_status lbm_batch_create(const lbm_handle *members, int32_t n, void *stream, lbm_batch *out)
{
    if (!members || n < 1 || !out) return LBM_ERR_ARG;
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        lbm_ctx *h = members[i];
        if (!h) return LBM_ERR_ARG;
        if (!h->initialized) return fail(h, LBM_ERR_STATE, "batch member %d: lbm_init_fields has not been called", i);
        if (h->dirty) return fail(h, LBM_ERR_STATE, "batch member %d: bodies set since the last step", i);
        if (h->cfg.storage != members[0]->cfg.storage)
            return fail(h, LBM_ERR_ARG, "batch member %d: storage differs from member 0", i);
        if (h->zieb_z >= 0) return fail(h, LBM_ERR_ARG, "batch member %d has an inflow plane", i);
        for (int j = 0; j < i; ++j)
            if (members[j] == h) return fail(h, LBM_ERR_ARG, "batch member %d repeats member %d", i, j);
    }
    lbm_batch_ctx *b = new (std::nothrow) lbm_batch_ctx();
    if (!b) return LBM_ERR_OOM;
    b->m.assign(members, members + n);
    b->storage = members[0]->cfg.storage;
    b->shape = kTile32x4x2;
    bool all64 = true;
    for (lbm_ctx *h : b->m) all64 = all64 && h->cfg.nx % 64 == 0;
    if (all64) b->shape = kTile64x2x2;
    if (stream) {
        b->stream = (hipStream_t)stream;
    } else if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) == hipSuccess) {
        b->own_stream = true;
    } else {
        delete b;
        return LBM_ERR_HIP;
    }
    for (lbm_ctx *h : b->m)
        if (hipStreamSynchronize(h->stream) != hipSuccess) {
            lbm_batch_destroy(b);
            return LBM_ERR_HIP;
        }
    const lbm_status st = batch_build(b);
    if (st != LBM_OK) {
        for (lbm_ctx *h : b->m) h->err = "lbm_batch_create: " + b->err;
        lbm_batch_destroy(b);
        return st;
    }
    *out = b;
    return LBM_OK;
}

}  // extern "C"

namespace {

// Wait for the members' queued work and load their state parities.  A
// member whose geometry or state was replaced since the batch was built
// (bodies set, stepped, state restored) is refused: the captured graphs hold
// its old tables.
lbm_status batch_sync_members(lbm_batch_ctx *b)
{
    const int n = (int)b->m.size();
    for (int i = 0; i < n; ++i) {
        lbm_ctx *h = b->m[(size_t)i];
        if (h->dirty) return bfail(b, LBM_ERR_STATE, "member %d: bodies set since the batch was built", i);
        if (h->geom_gen != b->gen[(size_t)i])
            return bfail(b, LBM_ERR_STATE, "member %d: geometry or state replaced since the batch was built", i);
        if (finish_forces(h, nullptr) != LBM_OK) return bfail(b, LBM_ERR_HIP, "member %d: %s", i, h->err.c_str());
        BHIP_TRY(b, hipStreamSynchronize(h->stream));
        b->h_cur[i] = h->cur;
    }
    BHIP_TRY(b, hipMemcpyAsync(b->d_cur, b->h_cur, sizeof(int) * (size_t)n, hipMemcpyHostToDevice, b->stream));
    return LBM_OK;
}

// Clear the members' force sums (after launches that only time the kernel).
lbm_status batch_zero_sums(lbm_batch_ctx *b)
{
    for (lbm_ctx *h : b->m) BHIP_TRY(b, launch_zero_fix(h->fsum[h->fcur], (int)fsum_entries(h->cfg), b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_batch_set_tile(lbm_batch b, int32_t shape)
{
    if (!b) return LBM_ERR_ARG;
    if (shape < 0 || shape >= kNumTileShapes) return bfail(b, LBM_ERR_ARG, "tile shape %d out of range", shape);
    b->shape = shape;
    return batch_build(b);
}

lbm_status lbm_batch_get_tile(lbm_batch b, int32_t *shape)
{
    if (!b || !shape) return b ? bfail(b, LBM_ERR_ARG, "NULL output") : LBM_ERR_ARG;
    *shape = b->shape;
    return LBM_OK;
}

lbm_status lbm_batch_autotune(lbm_batch b, int32_t trial_steps, int32_t *shape_out, double *us)
{
    if (!b) return LBM_ERR_ARG;
    if (trial_steps < 1) return bfail(b, LBM_ERR_ARG, "trial_steps < 1");
    if (us)
        for (int k = 0; k < kNumTileShapes; ++k) us[k] = -1.0;
    lbm_status st = batch_sync_members(b);
    if (st != LBM_OK) return st;
    // the batched step kernel reads every member's current state and writes
    // only the spare buffers and the force sums (cleared afterwards):
    // repeated launches leave the states as they are
    // two passes over the shapes, each shape's best pass kept (as for one
    // lattice: the first trials of a GPU that has just started run slow)
    EventPair ev;
    BHIP_TRY(b, ev.create());
    double t_best[kNumTileShapes];
    for (int pass = 0; pass < 2; ++pass)
        for (int k = 0; k < kNumTileShapes; ++k) {
            b->shape = k;
            if ((st = batch_build(b)) != LBM_OK) return st;
            // each launch followed by the reset of the tile queues (a flip of no member)
            BHIP_TRY(b, launch_batch_step(b->storage, k, b->bs, b->grid_step, b->stream));
            BHIP_TRY(b, launch_batch_flip(b->d_cur, 0, b->d_queue, b->stream));
            BHIP_TRY(b, hipEventRecord(ev.e0, b->stream));
            for (int i = 0; i < trial_steps; ++i) {
                BHIP_TRY(b, launch_batch_step(b->storage, k, b->bs, b->grid_step, b->stream));
                BHIP_TRY(b, launch_batch_flip(b->d_cur, 0, b->d_queue, b->stream));
            }
            BHIP_TRY(b, hipEventRecord(ev.e1, b->stream));
            BHIP_TRY(b, hipEventSynchronize(ev.e1));
            float ms = 0.f;
            BHIP_TRY(b, hipEventElapsedTime(&ms, ev.e0, ev.e1));
            const double t = 1e3 * ms / trial_steps;
            t_best[k] = pass == 0 ? t : std::min(t_best[k], t);
        }
    int best = 0;
    for (int k = 0; k < kNumTileShapes; ++k) {
        if (us) us[k] = t_best[k];
        if (t_best[k] < t_best[best]) best = k;
    }
    if ((st = batch_zero_sums(b)) != LBM_OK) return st;
    b->shape = best;
    if (shape_out) *shape_out = best;
    return batch_build(b);
}

lbm_status lbm_batch_step(lbm_batch b, int32_t nsteps)
{
    if (!b) return LBM_ERR_ARG;
    if (nsteps < 0) return bfail(b, LBM_ERR_ARG, "nsteps < 0");
    lbm_status st = batch_sync_members(b);
    if (st != LBM_OK) return st;
    for (int s = 0; s + kBatchBlock <= nsteps; s += kBatchBlock) BHIP_TRY(b, hipGraphLaunch(b->execB, b->stream));
    for (int s = 0; s < nsteps % kBatchBlock; ++s) BHIP_TRY(b, hipGraphLaunch(b->exec1, b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    for (lbm_ctx *h : b->m) {
        h->cur ^= nsteps & 1;
        h->steps_done += nsteps;
    }
    return LBM_OK;
}

}  // extern "C"
