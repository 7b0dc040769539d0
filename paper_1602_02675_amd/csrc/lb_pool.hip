// Pool runtime behind the lb_pool_* calls of include/lbsd.h: many independent
// problems (same lattice, gamma and precision; own grid, lambda, boundary
// conditions and step target) resident in one arena of the caller's device
// memory, advanced together by one persistent launch per step.
//
// Device-resident tables (rewritten by the host between launches, read by the
// kernels): one PoolProb per slot and the tile table (slot, first column,
// first row, rows).  The kernels never see the host's view of which slots are
// live: admissions and releases only rewrite the tables, so the launch shape,
// and a captured HIP graph of it, stay valid.  Each slot counts its own steps
// on the device (PoolState.done), which also selects its ping-pong moment set.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <vector>

#include "lb_host.hpp"

using namespace lbsd;

namespace {

struct SlotInfo {
    lb_grid grid;
    double lambda = 0.0;
    size_t arena_off = 0, bytes = 0;  // byte range in the arena
    int64_t target = 0;
};

// Pinned staging of one table upload; `ev` marks when the copies out of it
// have run.
struct Stage {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
};

// One progress snapshot (lb_pool_snapshot): the slot states copied behind the
// queued work into pinned memory, and the host's view of the slots when it
// was queued (admission count, target, lambda).
struct Snap {
    PoolState* host = nullptr;
    hipEvent_t ev = nullptr;
    bool queued = false;
    std::vector<int64_t> gen, target;
    std::vector<double> lambda;
};

}  // namespace

struct lb_pool {
    int dim = 0, nf = 0, precision = 0;
    size_t elem = 0;
    double gamma = 0.0, gamma2 = 0.0;  // gamma2: gas 2 (two gases), else gamma
    bool species = false;              // two gases: a species field rho chi after rho E
    lb_velset vs{};
    Consts k{};
    int32_t max_slots = 0;
    size_t arena_bytes = 0;
    int64_t max_tiles = 0;
    // layout inside the bound buffer
    size_t off_probs = 0, off_state = 0, off_tiles = 0, off_tstate = 0, off_ntiles = 0, off_partials = 0,
           off_flags = 0, off_arena = 0, total = 0;
    char* base = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false;
    int cus = 0;
    // host view
    std::vector<PoolProb> probs;
    std::vector<SlotInfo> info;
    std::map<size_t, size_t> free_list;  // arena byte offset -> size
    std::vector<PoolTile> tiles;
    int shape = 0;    // 1-D: kernel tile shape; 2-D: strip height index
    int nblocks = 0;  // persistent blocks of the current shape (square lattice: short and full passes)
    int nblocks_lean = 0;  // square lattice: persistent blocks of the lean pass
    bool walls = false;  // a live slot has reflecting walls: run the kernels that handle them
    // graph of `graph_steps` steps (0: plain launches)
    int graph_steps = 0;
    bool graph_ready = false;
    hipGraphExec_t graph_exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // stream-ordered table uploads (two stagings used in turn) and snapshots
    Stage stage[2];
    int stage_next = 0;
    Snap snap[2];
    std::vector<int64_t> gen;  // admissions per slot
    bool dirty = false;        // the tables changed since the last upload (sent before the next step)
};

namespace {

PoolView view_of(const lb_pool* p)
{
    PoolView v;
    v.probs = (const PoolProb*)(p->base + p->off_probs);
    v.state = (PoolState*)(p->base + p->off_state);
    v.tiles = (const PoolTile*)(p->base + p->off_tiles);
    v.tstate = (int32_t*)(p->base + p->off_tstate);
    v.ntiles = (const int32_t*)(p->base + p->off_ntiles);
    v.partials = (double*)(p->base + p->off_partials);
    v.flags = (int32_t*)(p->base + p->off_flags);
    v.flags_lean = v.flags + p->max_tiles;
    v.next = (int32_t*)(p->base + p->off_ntiles + 64);
    v.arena = p->base + p->off_arena;
    return v;
}

size_t set_bytes(const lb_pool* p, int64_t nn) { return align256((size_t)p->nf * (size_t)nn * p->elem); }

int64_t tile_cols(const lb_pool* p) { return p->dim == 1 ? (int64_t)kPool1TPB[p->shape] * kPool1J[p->shape] : kPool2Cols; }
int64_t tiles_of(const lb_pool* p, int64_t nx, int64_t ny, int shape)
{
    if (p->dim == 1) {
        const int64_t t = (int64_t)kPool1TPB[shape] * kPool1J[shape];
        return (nx + t - 1) / t;
    }
    return ((nx + kPool2Cols - 1) / kPool2Cols) * ((ny + kPool2MinRows - 1) / kPool2MinRows);  // at most
}

int launch_blocks(const lb_pool* p, int64_t ntiles, bool lean = false);

// Rows per tile: 1 in 1-D; on the square lattice about
// kPool2TilesPerBlock[shape] tiles per resident block over the live problems.
int64_t tile_rows(const lb_pool* p)
{
    if (p->dim == 1) return 1;
    int64_t strip_rows = 0;  // rows of all column strips of the live problems
    for (int i = 0; i < p->max_slots; ++i) {
        const PoolProb& q = p->probs[(size_t)i];
        if (q.active) strip_rows += ((q.nx + kPool2Cols - 1) / kPool2Cols) * q.ny;
    }
    const int64_t want = (int64_t)kPool2TilesPerBlock[p->shape] * launch_blocks(p, 0, true);
    const int64_t rows = (strip_rows + want - 1) / std::max<int64_t>(want, 1);
    return std::max<int64_t>(rows, kPool2MinRows);
}

// Worst case over the shapes, so that a later shape change always fits.
int64_t max_tiles_of(const lb_pool* p, int64_t nx, int64_t ny)
{
    int64_t m = 0;
    const int ns = p->dim == 1 ? kPool1Shapes : kPool2Shapes;
    for (int s = 0; s < ns; ++s) m = std::max(m, tiles_of(p, nx, ny, s));
    return m;
}

int64_t live_max_tiles(const lb_pool* p)
{
    int64_t n = 0;
    for (int i = 0; i < p->max_slots; ++i)
        if (p->probs[i].active) n += max_tiles_of(p, p->probs[i].nx, p->probs[i].ny);
    return n;
}

// Blocks of the step launch.  Square lattice: persistent blocks (as many as
// are resident at once) that claim tiles, so that slow tiles spread out.  1-D:
// one block per tile (tiles cost about the same, and the hardware then
// overlaps one tile's loads with other tiles' work).
int launch_blocks(const lb_pool* p, int64_t ntiles, bool lean)
{
    if (p->dim == 1) return (int)std::max<int64_t>(1, ntiles);
    const int per_cu = p->precision == LB_FP64 ? pool2d_blocks_per_cu<double>(lean) : pool2d_blocks_per_cu<float>(lean);
    return std::max(1, p->cus * per_cu);
}

void drop_graph(lb_pool* p)
{
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    p->graph_exec = nullptr;
    p->graph_ready = false;
}

// Per-tile word from the device's slot states: the set holding the slot's
// moments, and whether the slot still steps.
__global__ void pool_tile_words_kernel(PoolView v, int32_t nt)
{
    const int32_t t = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= nt) return;
    const int32_t i = v.tiles[t].prob;
    const PoolState& q = v.state[i];
    v.tstate[t] = (int32_t)(q.done & 1) | (q.err_step == 0 && q.done < v.probs[i].target ? kTileLive : 0);
}

// A fresh state record for a slot being admitted.
__global__ void pool_reset_state_kernel(PoolState* st)
{
    if (threadIdx.x == 0) *st = PoolState{};
}

// Rebuild the tile table of the live slots (slot order, then rows, then
// columns) and queue its upload with the slot table on the pool's stream:
// the kernels of steps queued earlier still see the old tables, those queued
// later the new ones.  The host returns at once (it waits only when both
// pinned stagings still have copies in flight).
int upload_tables(lb_pool* p)
{
    p->tiles.clear();
    const int64_t tc = tile_cols(p), tr = tile_rows(p);
    for (int i = 0; i < p->max_slots; ++i) {
        PoolProb& q = p->probs[i];
        q.t0 = (int64_t)p->tiles.size();
        if (q.active) {
            for (int64_t y0 = 0; y0 < q.ny; y0 += tr)
                for (int64_t x0 = 0; x0 < q.nx; x0 += tc) {
                    PoolTile t;
                    t.prob = i;
                    t.rows = (int32_t)tr;
                    t.x0 = x0;
                    t.y0 = y0;
                    t.off[0] = q.off[0];
                    t.off[1] = q.off[1];
                    t.nx = q.nx;
                    t.ny = q.ny;
                    t.bc_x = q.bc_x;
                    t.bc_y = q.bc_y;
                    p->tiles.push_back(t);
                }
        }
        q.t1 = (int64_t)p->tiles.size();
    }
    if ((int64_t)p->tiles.size() > p->max_tiles) return fail(LB_ENOMEM, "tile table full");
    const int32_t nt = (int32_t)p->tiles.size();
    const int nb = launch_blocks(p, nt), nb_lean = launch_blocks(p, nt, true);
    bool walls = false;
    for (const PoolProb& q : p->probs)
        walls |= q.active && (q.bc_x == kBcReflecting || (p->dim == 2 && q.bc_y == kBcReflecting));
    if (nb != p->nblocks || nb_lean != p->nblocks_lean || walls != p->walls) {  // a captured graph is stale
        drop_graph(p);
        p->nblocks = nb;
        p->nblocks_lean = nb_lean;
        p->walls = walls;
    }
    // probs, tile count and tiles through a pinned staging
    const size_t pb = p->probs.size() * sizeof(PoolProb), tb = (size_t)nt * sizeof(PoolTile);
    const size_t at_nt = align256(pb), at_tiles = at_nt + 256, need = at_tiles + tb;
    Stage& sg = p->stage[p->stage_next];
    p->stage_next ^= 1;
    hipError_t e;
    if (sg.pending) {
        if ((e = hipEventSynchronize(sg.ev)) != hipSuccess) return hip_fail(e, "staging wait");
        sg.pending = false;
    }
    if (sg.cap < need) {
        if (sg.host) (void)hipHostFree(sg.host);
        sg.host = nullptr;
        sg.cap = 0;
        if ((e = hipHostMalloc(&sg.host, need, hipHostMallocDefault)) != hipSuccess)
            return hip_fail(e, "pinned staging");
        sg.cap = need;
    }
    char* h = (char*)sg.host;
    memcpy(h, p->probs.data(), pb);
    memcpy(h + at_nt, &nt, sizeof nt);
    if (nt > 0) memcpy(h + at_tiles, p->tiles.data(), tb);
    if ((e = hipMemcpyAsync(p->base + p->off_probs, h, pb, hipMemcpyHostToDevice, p->stream)) != hipSuccess)
        return hip_fail(e, "upload slots");
    if (nt > 0 && (e = hipMemcpyAsync(p->base + p->off_tiles, h + at_tiles, tb, hipMemcpyHostToDevice,
                                      p->stream)) != hipSuccess)
        return hip_fail(e, "upload tiles");
    if ((e = hipMemcpyAsync(p->base + p->off_ntiles, h + at_nt, sizeof nt, hipMemcpyHostToDevice, p->stream)) !=
        hipSuccess)
        return hip_fail(e, "upload tile count");
    if ((e = hipEventRecord(sg.ev, p->stream)) != hipSuccess) return hip_fail(e, "staging event");
    sg.pending = true;
    // claim counters and tile flags cleared; tile words from the slots' device states
    const PoolView v = view_of(p);
    if ((e = launch_fill_i32(v.next, 5, 0, p->stream)) != hipSuccess) return hip_fail(e, "clear claim counters");
    if (nt > 0 && (e = launch_fill_i32(v.flags, nt, 0, p->stream)) != hipSuccess) return hip_fail(e, "clear flags");
    if (nt > 0 && p->dim == 2 && (e = launch_fill_i32(v.flags_lean, nt, 0, p->stream)) != hipSuccess)
        return hip_fail(e, "clear lean flags");
    if (nt > 0) {
        pool_tile_words_kernel<<<(unsigned)((nt + 255) / 256), 256, 0, p->stream>>>(v, nt);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "tile words");
    }
    return LB_OK;
}

int set_shape(lb_pool* p, int shape)
{
    const int ns = p->dim == 1 ? kPool1Shapes : kPool2Shapes;
    if (shape < 0 || shape >= ns) return fail(LB_EINVAL, "shape must lie in [0, %d)", ns);
    if (shape != p->shape) drop_graph(p);
    p->shape = shape;
    const int rc = upload_tables(p);
    if (rc == LB_OK) p->dirty = false;
    return rc;
}

// One step of every live slot: step kernel(s), then the per-slot reduction.
int queue_step(lb_pool* p, int commit)
{
    const PoolView v = view_of(p);
    hipError_t e;
    if (p->dim == 1)
        e = p->precision == LB_FP64 ? launch_pool1d<double>(v, p->k, p->shape, p->nblocks, p->walls, p->stream)
                                    : launch_pool1d<float>(v, p->k, p->shape, p->nblocks, p->walls, p->stream);
    else
        e = p->precision == LB_FP64
            ? launch_pool2d<double>(v, p->k, p->nblocks_lean, p->nblocks, p->walls, p->stream)
            : launch_pool2d<float>(v, p->k, p->nblocks_lean, p->nblocks, p->walls, p->stream);
    if (e != hipSuccess) return hip_fail(e, "pool step launch");
    if ((e = launch_pool_finalize(v, p->max_slots, commit, p->stream)) != hipSuccess)
        return hip_fail(e, "pool finalize launch");
    return LB_OK;
}

int capture_graph(lb_pool* p)
{
    drop_graph(p);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    int rc = LB_OK;
    for (int i = 0; i < p->graph_steps && rc == LB_OK; ++i) rc = queue_step(p, 1);
    e = hipStreamEndCapture(p->stream, &graph);
    if (rc != LB_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&p->graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        p->graph_exec = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    p->graph_ready = true;
    return LB_OK;
}

int flush_tables(lb_pool* p);

int queue_steps(lb_pool* p, int64_t n)
{
    int rc0 = flush_tables(p);  // never inside a captured graph
    if (rc0 != LB_OK) return rc0;
    int64_t left = n;
    if (p->graph_steps > 0 && left >= p->graph_steps) {
        if (!p->graph_ready) {
            const int rc = capture_graph(p);
            if (rc != LB_OK) return rc;
        }
        for (; left >= p->graph_steps; left -= p->graph_steps) {
            hipError_t e = hipGraphLaunch(p->graph_exec, p->stream);
            if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        }
    }
    for (; left > 0; --left) {
        const int rc = queue_step(p, 1);
        if (rc != LB_OK) return rc;
    }
    return LB_OK;
}

int read_state(lb_pool* p, int32_t slot, PoolState* st)
{
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "sync");
    e = hipMemcpy(st, p->base + p->off_state + (size_t)slot * sizeof(PoolState), sizeof *st,
                  hipMemcpyDeviceToHost);
    return e == hipSuccess ? LB_OK : hip_fail(e, "read slot state");
}

int check_slot(const lb_pool* p, int32_t slot)
{
    if (!p || !p->bound) return fail(LB_EINVAL, "pool not bound");
    if (slot < 0 || slot >= p->max_slots || !p->probs[(size_t)slot].active)
        return fail(LB_EINVAL, "slot %d is not admitted", slot);
    return LB_OK;
}

// First fit in the arena's free list.
bool arena_take(lb_pool* p, size_t bytes, size_t* off)
{
    for (auto it = p->free_list.begin(); it != p->free_list.end(); ++it) {
        if (it->second < bytes) continue;
        *off = it->first;
        const size_t rest = it->second - bytes, at = it->first + bytes;
        p->free_list.erase(it);
        if (rest > 0) p->free_list[at] = rest;
        return true;
    }
    return false;
}

void arena_give(lb_pool* p, size_t off, size_t bytes)
{
    auto it = p->free_list.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != p->free_list.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        p->free_list.erase(nx);
    }
    if (it != p->free_list.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            p->free_list.erase(it);
        }
    }
}

// Reserve a slot and arena space for a grid; fills probs/info (inactive until
// the state is written).  LB_ENOMEM when it does not fit now.
int reserve(lb_pool* p, const lb_grid* grid, int64_t steps, int32_t* slot_out)
{
    if (!p || !p->bound) return fail(LB_EINVAL, "pool not bound");
    int rc = check_grid(grid, p->dim);
    if (rc != LB_OK) return rc;
    if (steps < 0) return fail(LB_EINVAL, "steps must be >= 0");
    int32_t slot = -1;
    for (int32_t i = 0; i < p->max_slots; ++i)
        if (!p->probs[(size_t)i].active) { slot = i; break; }
    if (slot < 0) return fail(LB_ENOMEM, "no free slot (%d in use)", p->max_slots);
    const int64_t nn = grid->nx * grid->ny;
    if (live_max_tiles(p) + max_tiles_of(p, grid->nx, grid->ny) > p->max_tiles)
        return fail(LB_ENOMEM, "tile table full");
    const size_t sb = set_bytes(p, nn), bytes = 2 * sb;
    size_t off = 0;
    if (!arena_take(p, bytes, &off))
        return fail(LB_ENOMEM, "%zu arena bytes needed, no free block that large", bytes);
    PoolProb& q = p->probs[(size_t)slot];
    q = PoolProb{};
    q.off[0] = (int64_t)(off / p->elem);
    q.off[1] = (int64_t)((off + sb) / p->elem);
    q.nx = grid->nx;
    q.ny = grid->ny;
    q.bc_x = grid->bc_x;
    q.bc_y = grid->bc_y;
    q.target = steps;
    SlotInfo& si = p->info[(size_t)slot];
    si.grid = *grid;
    si.arena_off = off;
    si.bytes = bytes;
    si.target = steps;
    *slot_out = slot;
    return LB_OK;
}

void unreserve(lb_pool* p, int32_t slot)
{
    PoolProb& q = p->probs[(size_t)slot];
    arena_give(p, p->info[(size_t)slot].arena_off, p->info[(size_t)slot].bytes);
    q = PoolProb{};
}

// Make a reserved slot live: fresh state record, tables uploaded (both
// stream-ordered behind the work queued so far).
int activate(lb_pool* p, int32_t slot)
{
    pool_reset_state_kernel<<<1, 64, 0, p->stream>>>((PoolState*)(p->base + p->off_state) + slot);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "reset slot state");
    p->probs[(size_t)slot].active = 1;
    p->gen[(size_t)slot] += 1;
    p->dirty = true;
    return LB_OK;
}

// Send the tables if admissions or releases changed them (before a step).
int flush_tables(lb_pool* p)
{
    if (!p->dirty) return LB_OK;
    const int rc = upload_tables(p);
    if (rc == LB_OK) p->dirty = false;
    return rc;
}

void* set_ptr(const lb_pool* p, int32_t slot, int set)
{
    return p->base + p->off_arena + (size_t)p->probs[(size_t)slot].off[set] * p->elem;
}

}  // namespace

extern "C" {

static int create_pool(int32_t dim, double gamma, double gamma2, bool species, const lb_velset* vs,
                       int32_t precision, int32_t max_slots, size_t arena_bytes, lb_pool** out)
{
    if (!vs || !out) return fail(LB_EINVAL, "null argument");
    int rc = check_model(dim, gamma, vs, precision);
    if (rc != LB_OK) return rc;
    if (species && (rc = check_model(dim, gamma2, vs, precision)) != LB_OK) return rc;
    if (is_hex(vs)) return fail(LB_EINVAL, "pools run the 1-D and square lattices");
    if (max_slots < 1 || max_slots > (1 << 20)) return fail(LB_EINVAL, "max_slots must lie in [1, 2^20]");
    if (arena_bytes < 256) return fail(LB_EINVAL, "arena too small");
    lb_pool* p = new (std::nothrow) lb_pool();
    if (!p) return fail(LB_ENOMEM, "host allocation failed");
    p->dim = dim;
    p->species = species;
    p->nf = dim + 2 + (species ? 1 : 0);
    p->precision = precision;
    p->elem = precision == LB_FP64 ? 8 : 4;
    p->gamma = gamma;
    p->gamma2 = species ? gamma2 : gamma;
    p->vs = *vs;
    p->k = make_consts(dim, gamma, vs);
    p->k.g1m1 = gamma - 1.0;
    p->k.g2m1 = p->gamma2 - 1.0;
    p->k.species = species ? 1 : 0;
    p->max_slots = max_slots;
    p->arena_bytes = arena_bytes & ~(size_t)255;
    // every live slot has at most one partly filled tile row/column per
    // shape; the rest of its tiles are full (>= 256 nodes in 1-D, >= 246 x 16
    // on the square lattice)
    const int64_t cap_nodes = (int64_t)(p->arena_bytes / (2 * (size_t)p->nf * p->elem));
    p->max_tiles = (int64_t)max_slots * (dim == 1 ? 1 : 64) + cap_nodes / (dim == 1 ? 256 : 246) + 64;
    try {
        p->probs.assign((size_t)max_slots, PoolProb{});
        p->info.assign((size_t)max_slots, SlotInfo{});
        p->gen.assign((size_t)max_slots, 0);
    } catch (...) {
        delete p;
        return fail(LB_ENOMEM, "host allocation failed");
    }
    p->shape = dim == 1 ? 2 : 3;  // 1024-node tiles / 128-row strips until tuned
    p->off_probs = 0;
    p->off_state = align256((size_t)max_slots * sizeof(PoolProb));
    p->off_tiles = p->off_state + align256((size_t)max_slots * sizeof(PoolState));
    p->off_tstate = p->off_tiles + align256((size_t)p->max_tiles * sizeof(PoolTile));
    p->off_ntiles = p->off_tstate + align256((size_t)p->max_tiles * 4);
    p->off_partials = p->off_ntiles + 256;  // tile count at +0, claim counters at +64
    p->off_flags = p->off_partials + align256((size_t)p->max_tiles * kPartialStride * 8);
    p->off_arena = p->off_flags + align256((size_t)p->max_tiles * 2 * 4);  // two flag words per tile
    p->total = p->off_arena + p->arena_bytes;
    p->free_list[0] = p->arena_bytes;
    *out = p;
    return LB_OK;
}

int lb_pool_create(int32_t dim, double gamma, const lb_velset* vs, int32_t precision, int32_t max_slots,
                   size_t arena_bytes, lb_pool** out)
{
    return create_pool(dim, gamma, gamma, false, vs, precision, max_slots, arena_bytes, out);
}

int lb_pool_create_two_gas(int32_t dim, double gamma_1, double gamma_2, const lb_velset* vs, int32_t precision,
                           int32_t max_slots, size_t arena_bytes, lb_pool** out)
{
    return create_pool(dim, gamma_1, gamma_2, true, vs, precision, max_slots, arena_bytes, out);
}

size_t lb_pool_bytes(const lb_pool* p) { return p ? p->total : 0; }

size_t lb_pool_footprint(const lb_pool* p, int64_t nx, int64_t ny)
{
    if (!p || nx < 1 || ny < 1) return 0;
    return 2 * set_bytes(p, nx * ny);
}

int lb_pool_bind(lb_pool* p, void* dev_ptr, size_t bytes, void* hip_stream)
{
    if (!p || !dev_ptr) return fail(LB_EINVAL, "null argument");
    if (p->bound) return fail(LB_EINVAL, "pool already bound");
    if (bytes < p->total) return fail(LB_ENOMEM, "buffer of %zu bytes < %zu needed", bytes, p->total);
    if ((uintptr_t)dev_ptr % 256 != 0) return fail(LB_EINVAL, "device buffer must be 256-byte aligned");
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, dev_ptr);
    if (e != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return fail(LB_EINVAL, "pointer is not device memory");
    }
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
    if ((e = hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return hip_fail(e, "hipDeviceGetAttribute");
    if ((e = hipEventCreate(&p->ev0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&p->ev1)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    for (Stage& sg : p->stage)
        if ((e = hipEventCreateWithFlags(&sg.ev, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    for (Snap& sn : p->snap) {
        if ((e = hipEventCreateWithFlags(&sn.ev, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "hipEventCreate");
        if ((e = hipHostMalloc((void**)&sn.host, (size_t)p->max_slots * sizeof(PoolState), hipHostMallocDefault)) !=
            hipSuccess)
            return hip_fail(e, "pinned snapshot");
    }
    p->base = (char*)dev_ptr;
    p->stream = (hipStream_t)hip_stream;
    p->bound = true;
    // zero slot states, then the (empty) tables
    static_assert(sizeof(PoolState) % 4 == 0, "slot states are cleared as 32-bit words");
    if ((e = launch_fill_i32((int32_t*)(p->base + p->off_state), (int64_t)p->max_slots * sizeof(PoolState) / 4, 0,
                             p->stream)) != hipSuccess)
        return hip_fail(e, "clear slot states");
    const int rc = set_shape(p, p->shape);
    if (rc != LB_OK) return rc;
    if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return hip_fail(e, "sync");
    return LB_OK;
}

int lb_pool_admit_riemann(lb_pool* p, const lb_grid* grid, double lambda, double x_d, const lb_prim* L,
                          const lb_prim* R, int64_t steps, int32_t* slot)
{
    if (!slot) return fail(LB_EINVAL, "null slot");
    if (!isfinite(x_d)) return fail(LB_EINVAL, "diaphragm position must be finite");
    if (!p) return fail(LB_EINVAL, "null pool");
    double lam = 0.0, side[2][5];
    int rc = riemann_sides(p->dim, p->gamma, p->gamma2, p->species, lambda, 1.0, L, R, &lam, side);
    if (rc != LB_OK) return rc;
    int32_t s = -1;
    if ((rc = reserve(p, grid, steps, &s)) != LB_OK) return rc;
    const Grid g{grid->nx, grid->ny, grid->bc_x, grid->bc_y};
    const double dx = (grid->x_hi - grid->x_lo) / (double)grid->nx;
    hipError_t e = p->precision == LB_FP64
        ? launch_init_riemann<double>((double*)set_ptr(p, s, 0), g, p->nf, grid->x_lo, dx, x_d, side[0], side[1],
                                      p->stream)
        : launch_init_riemann<float>((float*)set_ptr(p, s, 0), g, p->nf, grid->x_lo, dx, x_d, side[0], side[1],
                                     p->stream);
    if (e != hipSuccess) {
        unreserve(p, s);
        return hip_fail(e, "init kernel");
    }
    p->info[(size_t)s].lambda = lam;
    if ((rc = activate(p, s)) != LB_OK) {
        unreserve(p, s);
        return rc;
    }
    *slot = s;
    return LB_OK;
}

int lb_pool_admit_moments(lb_pool* p, const lb_grid* grid, const double* host_Y, double lambda, int64_t steps,
                          int32_t* slot)
{
    if (!p || !slot || !grid) return fail(LB_EINVAL, "null argument");
    if (!(lambda > 0.0) || !isfinite(lambda)) return fail(LB_EINVAL, "lambda must be > 0");
    int rc = check_grid(grid, p->dim);
    if (rc != LB_OK) return rc;
    if ((rc = check_moments(host_Y, p->nf, grid->nx * grid->ny)) != LB_OK) return rc;
    if (p->species && (rc = check_species(host_Y, p->nf, grid->nx * grid->ny)) != LB_OK) return rc;
    int32_t s = -1;
    if ((rc = reserve(p, grid, steps, &s)) != LB_OK) return rc;
    rc = upload_moments(set_ptr(p, s, 0), host_Y, p->nf, p->dim + 1, grid->nx * grid->ny, lambda,
                        p->precision == LB_FP64,
                        p->stream);
    if (rc == LB_OK) {
        p->info[(size_t)s].lambda = lambda;
        rc = activate(p, s);
    }
    if (rc != LB_OK) {
        unreserve(p, s);
        return rc;
    }
    *slot = s;
    return LB_OK;
}

// No wait: steps queued earlier still run the released slot with the old
// tables; whatever reuses its memory (an admission's initial state) is
// queued after them on the same stream.
int lb_pool_release(lb_pool* p, int32_t slot)
{
    int rc = check_slot(p, slot);
    if (rc != LB_OK) return rc;
    unreserve(p, slot);
    return upload_tables(p);
}

int lb_pool_advance(lb_pool* p, int64_t n)
{
    if (!p || !p->bound) return fail(LB_EINVAL, "pool not bound");
    if (n < 0) return fail(LB_EINVAL, "n must be >= 0");
    return queue_steps(p, n);
}

int lb_pool_advance_timed(lb_pool* p, int64_t n, float* ms)
{
    if (!p || !p->bound || !ms) return fail(LB_EINVAL, "null argument or pool not bound");
    if (n < 0) return fail(LB_EINVAL, "n must be >= 0");
    {
        const int rc = flush_tables(p);  // outside the timed region
        if (rc != LB_OK) return rc;
    }
    if (p->graph_steps > 0 && !p->graph_ready && n >= p->graph_steps) {
        const int rc = capture_graph(p);  // outside the timed region
        if (rc != LB_OK) return rc;
    }
    hipError_t e;
    if ((e = hipEventRecord(p->ev0, p->stream)) != hipSuccess) return hip_fail(e, "event");
    int rc = queue_steps(p, n);
    if (rc != LB_OK) return rc;
    if ((e = hipEventRecord(p->ev1, p->stream)) != hipSuccess) return hip_fail(e, "event");
    if ((e = hipEventSynchronize(p->ev1)) != hipSuccess) return hip_fail(e, "event sync");
    float t = 0.f;
    if ((e = hipEventElapsedTime(&t, p->ev0, p->ev1)) != hipSuccess) return hip_fail(e, "elapsed");
    *ms = t;
    return LB_OK;
}

int lb_pool_poll(lb_pool* p, int32_t slot, int64_t* steps_done, int32_t* status)
{
    int rc = check_slot(p, slot);
    if (rc != LB_OK) return rc;
    PoolState st;
    if ((rc = read_state(p, slot, &st)) != LB_OK) return rc;
    if (steps_done) *steps_done = st.done;
    if (status) {
        if (st.err_step != 0) *status = (st.err_code & kErrState) ? LB_ESTATE : LB_EREACH;
        else *status = st.done >= p->probs[(size_t)slot].target ? 1 : 0;
    }
    return LB_OK;
}

int lb_pool_status(lb_pool* p, int64_t* steps_done, int32_t* status)
{
    if (!p || !p->bound) return fail(LB_EINVAL, "pool not bound");
    if (!steps_done || !status) return fail(LB_EINVAL, "null argument");
    std::vector<PoolState> st;
    try { st.resize((size_t)p->max_slots); } catch (...) { return fail(LB_ENOMEM, "host allocation failed"); }
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "sync");
    e = hipMemcpy(st.data(), p->base + p->off_state, st.size() * sizeof(PoolState), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read slot states");
    for (int32_t i = 0; i < p->max_slots; ++i) {
        const PoolState& q = st[(size_t)i];
        if (!p->probs[(size_t)i].active) {
            steps_done[i] = 0;
            status[i] = -100;
            continue;
        }
        steps_done[i] = q.done;
        if (q.err_step != 0) status[i] = (q.err_code & kErrState) ? LB_ESTATE : LB_EREACH;
        else status[i] = q.done >= p->probs[(size_t)i].target ? 1 : 0;
    }
    return LB_OK;
}

int lb_pool_moments(lb_pool* p, int32_t slot, double* out, int32_t on_device)
{
    if (!out) return fail(LB_EINVAL, "null argument");
    int rc = check_slot(p, slot);
    if (rc != LB_OK) return rc;
    PoolState st;
    if ((rc = read_state(p, slot, &st)) != LB_OK) return rc;
    const SlotInfo& si = p->info[(size_t)slot];
    const int64_t nn = si.grid.nx * si.grid.ny;
    double sc[5];
    field_scales(p->nf, p->dim + 1, si.lambda, sc);
    const void* src = set_ptr(p, slot, (int)(st.done & 1));
    hipError_t e;
    if (on_device) {
        e = p->precision == LB_FP64 ? launch_export<double>((const double*)src, out, nn, p->nf, sc, p->stream)
                                    : launch_export<float>((const float*)src, out, nn, p->nf, sc, p->stream);
        if (e != hipSuccess) return hip_fail(e, "export kernel");
        if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return hip_fail(e, "sync");
        return LB_OK;
    }
    // host output: copy the raw set, convert with the export kernel's arithmetic
    const size_t n = (size_t)p->nf * (size_t)nn;
    std::vector<double> d;
    std::vector<float> f;
    try {
        if (p->precision == LB_FP64) d.resize(n);
        else f.resize(n);
    } catch (...) {
        return fail(LB_ENOMEM, "host allocation failed");
    }
    e = p->precision == LB_FP64 ? hipMemcpy(d.data(), src, n * 8, hipMemcpyDeviceToHost)
                                : hipMemcpy(f.data(), src, n * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "copy out");
    for (int fi = 0; fi < p->nf; ++fi)
        for (int64_t q = 0; q < nn; ++q) {
            const size_t i = (size_t)fi * nn + q;
            out[i] = (p->precision == LB_FP64 ? d[i] : (double)f[i]) / sc[fi];
        }
    return LB_OK;
}

int lb_pool_totals(lb_pool* p, int32_t slot, double out[4])
{
    if (!out) return fail(LB_EINVAL, "null argument");
    int rc = check_slot(p, slot);
    if (rc != LB_OK) return rc;
    PoolState st;
    if ((rc = read_state(p, slot, &st)) != LB_OK) return rc;
    if (st.done == 0 || st.totals_step != st.done) return fail(LB_EINVAL, "no completed step to report");
    double sc[5];
    field_scales(p->nf, p->dim + 1, p->info[(size_t)slot].lambda, sc);
    double o[4] = {0, 0, 0, 0};
    o[0] = st.totals[0] / sc[0];
    o[1] = st.totals[1] / sc[1];
    if (p->dim == 2) {
        o[2] = st.totals[2] / sc[2];
        o[3] = st.totals[3] / sc[3];
    } else {
        o[3] = st.totals[2] / sc[2];
    }
    for (int i = 0; i < 4; ++i) out[i] = o[i];
    return LB_OK;
}

double lb_pool_lambda(const lb_pool* p, int32_t slot)
{
    if (!p || slot < 0 || slot >= p->max_slots || !p->probs[(size_t)slot].active) return 0.0;
    return p->info[(size_t)slot].lambda;
}

int32_t lb_pool_live(const lb_pool* p)
{
    if (!p) return 0;
    int32_t n = 0;
    for (const PoolProb& q : p->probs) n += q.active ? 1 : 0;
    return n;
}

int32_t lb_pool_shapes(const lb_pool* p) { return p ? (p->dim == 1 ? kPool1Shapes : kPool2Shapes) : 0; }

int32_t lb_pool_shape(const lb_pool* p) { return p ? p->shape : -1; }

int lb_pool_set_shape(lb_pool* p, int32_t shape)
{
    if (!p || !p->bound) return fail(LB_EINVAL, "pool not bound");
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "sync");
    return set_shape(p, shape);
}

int lb_pool_autotune(lb_pool* p, int32_t trials, int32_t* best, float* ms_per_step)
{
    if (!p || !p->bound) return fail(LB_EINVAL, "pool not bound");
    if (trials < 1 || trials > 1000) return fail(LB_EINVAL, "trials must lie in [1, 1000]");
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "sync");
    const int ns = lb_pool_shapes(p), keep = p->shape;
    int arg = -1;
    float best_ms = 0.f;
    for (int s = 0; s < ns; ++s) {
        int rc = set_shape(p, s);
        if (rc != LB_OK) return rc;
        // trial steps read the current sets and write the other ones without
        // counting a step: the slots' states are unchanged
        if ((rc = queue_step(p, 0)) != LB_OK) return rc;  // warm-up
        std::vector<float> t((size_t)trials);
        for (int i = 0; i < trials; ++i) {
            if ((e = hipEventRecord(p->ev0, p->stream)) != hipSuccess) return hip_fail(e, "event");
            if ((rc = queue_step(p, 0)) != LB_OK) return rc;
            if ((e = hipEventRecord(p->ev1, p->stream)) != hipSuccess) return hip_fail(e, "event");
            if ((e = hipEventSynchronize(p->ev1)) != hipSuccess) return hip_fail(e, "event sync");
            if ((e = hipEventElapsedTime(&t[(size_t)i], p->ev0, p->ev1)) != hipSuccess)
                return hip_fail(e, "elapsed");
        }
        std::sort(t.begin(), t.end());
        const float med = t[t.size() / 2];
        if (arg < 0 || med < best_ms) {
            arg = s;
            best_ms = med;
        }
    }
    const int rc = set_shape(p, arg >= 0 ? arg : keep);
    if (rc != LB_OK) return rc;
    if (best) *best = arg;
    if (ms_per_step) *ms_per_step = best_ms;
    return LB_OK;
}

int lb_pool_use_graph(lb_pool* p, int32_t steps_per_graph)
{
    if (!p || !p->bound) return fail(LB_EINVAL, "pool not bound");
    if (steps_per_graph < 0 || steps_per_graph > 4096) return fail(LB_EINVAL, "steps_per_graph in [0, 4096]");
    if (steps_per_graph > 0 && p->stream == nullptr)
        return fail(LB_EINVAL, "HIP graph capture needs a non-default stream");
    drop_graph(p);
    p->graph_steps = steps_per_graph;
    return LB_OK;
}

int lb_pool_snapshot(lb_pool* p, int32_t buf)
{
    if (!p || !p->bound) return fail(LB_EINVAL, "pool not bound");
    if (buf < 0 || buf > 1) return fail(LB_EINVAL, "snapshot buffer must be 0 or 1");
    Snap& sn = p->snap[buf];
    hipError_t e;
    if (sn.queued && (e = hipEventSynchronize(sn.ev)) != hipSuccess) return hip_fail(e, "snapshot wait");
    if ((e = hipMemcpyAsync(sn.host, p->base + p->off_state, (size_t)p->max_slots * sizeof(PoolState),
                            hipMemcpyDeviceToHost, p->stream)) != hipSuccess)
        return hip_fail(e, "snapshot copy");
    if ((e = hipEventRecord(sn.ev, p->stream)) != hipSuccess) return hip_fail(e, "snapshot event");
    sn.gen = p->gen;
    sn.target.assign((size_t)p->max_slots, 0);
    sn.lambda.assign((size_t)p->max_slots, 0.0);
    for (int32_t i = 0; i < p->max_slots; ++i) {
        if (!p->probs[(size_t)i].active) sn.gen[(size_t)i] = -1;
        sn.target[(size_t)i] = p->probs[(size_t)i].target;
        sn.lambda[(size_t)i] = p->info[(size_t)i].lambda;
    }
    sn.queued = true;
    return LB_OK;
}

int lb_pool_snapshot_read(lb_pool* p, int32_t buf, int64_t* steps_done, int32_t* status, double* totals)
{
    if (!p || !p->bound) return fail(LB_EINVAL, "pool not bound");
    if (buf < 0 || buf > 1) return fail(LB_EINVAL, "snapshot buffer must be 0 or 1");
    if (!steps_done || !status) return fail(LB_EINVAL, "null argument");
    Snap& sn = p->snap[buf];
    if (!sn.queued) return fail(LB_EINVAL, "no snapshot queued in buffer %d", buf);
    hipError_t e = hipEventSynchronize(sn.ev);
    if (e != hipSuccess) return hip_fail(e, "snapshot wait");
    for (int32_t i = 0; i < p->max_slots; ++i) {
        const size_t u = (size_t)i;
        double* out = totals ? totals + 4 * u : nullptr;
        if (out) out[0] = out[1] = out[2] = out[3] = NAN;
        // free when queued, or admitted again since: not this occupant's progress
        if (sn.gen[u] < 0 || !p->probs[u].active || p->gen[u] != sn.gen[u]) {
            steps_done[i] = 0;
            status[i] = LB_POOL_FREE;
            continue;
        }
        const PoolState& q = sn.host[u];
        steps_done[i] = q.done;
        if (q.err_step != 0) status[i] = (q.err_code & kErrState) ? LB_ESTATE : LB_EREACH;
        else status[i] = q.done >= sn.target[u] ? 1 : 0;
        if (out && q.done > 0 && q.totals_step == q.done) {
            double sc[5];
            field_scales(p->nf, p->dim + 1, sn.lambda[u], sc);
            out[0] = q.totals[0] / sc[0];
            out[1] = q.totals[1] / sc[1];
            if (p->dim == 2) {
                out[2] = q.totals[2] / sc[2];
                out[3] = q.totals[3] / sc[3];
            } else {
                out[2] = 0.0;
                out[3] = q.totals[2] / sc[2];
            }
        }
    }
    return LB_OK;
}

void lb_pool_destroy(lb_pool* p)
{
    if (!p) return;
    if (p->bound) (void)hipStreamSynchronize(p->stream);
    drop_graph(p);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    for (Stage& sg : p->stage) {
        if (sg.host) (void)hipHostFree(sg.host);
        if (sg.ev) (void)hipEventDestroy(sg.ev);
    }
    for (Snap& sn : p->snap) {
        if (sn.host) (void)hipHostFree(sn.host);
        if (sn.ev) (void)hipEventDestroy(sn.ev);
    }
    delete p;
}

}  // extern "C"
