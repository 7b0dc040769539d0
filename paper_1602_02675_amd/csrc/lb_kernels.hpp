// Kernel-side interface shared by the step kernels and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lb_device.hpp"

namespace lbsd {

constexpr int kErrReach = 1;  // a packet would travel further than the halo
constexpr int kErrState = 2;  // rho <= 0 or a non-finite moment

// Per-solver control block in device memory (written by the step kernels).
struct StepCtl {
    int next[5];            // square lattice: tile claim counters of the short- and full-FIFO passes,
                            // tiles the short pass flagged, claim counter of the lean pass, tiles the
                            // lean pass gave up (reset by finalize)
    int err_code;           // kErr* bits of the first failed step
    long long err_step;     // first failed step (LLONG_MAX if none)
    long long totals_step;  // step whose totals are in `totals`
    double totals[4];       // interior sums of the moment fields (lattice units)
    int max_reach;          // largest reach seen in the latest step
    int redo_tiles;         // tiles the full-FIFO pass has recomputed since the last reset
    int keep[2];            // square lattice: tiles the full-FIFO pass left flagged in this step [0]
                            // and in the previous step [1] (finalize moves [0] to [1])
    double totals_sp;       // square lattice with two gases: interior sum of rho chi
    int split_n[2];         // square lattice: tiles listed for row chunks in the steps of each parity
                            // (finalize clears the next step's)
    int full_n;             // square lattice: tiles the short pass listed for the full pass (finalize
                            // clears it)
};

// Per-block partial results: 4 field sums, reach, error bits; the square
// lattice with two gases puts the sum of rho chi at index 6.
constexpr int kPartialStride = 8;

struct Grid {
    int64_t nx, ny;  // ny = 1 in 1-D
    int bc_x, bc_y;
};

// Launch the step kernel of a 1-D / 2-D problem (async on `stream`).  Y and
// Yn are SoA [nf][ny][nx] arrays of T; partials receives one kPartialStride
// row per block (step_blocks_1d / march2d_blocks give the count), which
// launch_finalize then reduces.
template <typename T>
hipError_t launch_step1d(const T* Y, T* Yn, const Grid& g, const Consts& k, StepCtl* ctl,
                         double* partials, long long step, hipStream_t stream);
int64_t step_blocks_1d(const Grid& g);

// Square lattice, column-march kernel (lb_march2d.hip).  The grid is cut into
// tiles (column strips x row chunks) that the device's resident blocks claim
// one after another.
struct MarchGeom {
    int sy;                   // destination rows per tile
    int64_t grid_x, grid_y;   // tiles along x (column strips) and y (row chunks)
    int nblocks;              // persistent blocks of the short and full passes (resident at once)
    int nblocks_lean;         // persistent blocks of the lean pass
    int64_t blocks() const { return grid_x * grid_y; }  // tiles (= rows of partials)
};
// cus: compute units; per_cu / per_cu_lean: resident blocks per CU of the
// short and the lean pass (march2d_blocks_per_cu).
MarchGeom march2d_geometry(const Grid& g, int cus, int per_cu, int per_cu_lean);
int64_t march2d_max_blocks(const Grid& g);
// Resident blocks per CU of the short pass (lean = false) or the lean pass.
template <typename T>
int march2d_blocks_per_cu(bool lean = false);
// The short-FIFO kernel runs every tile and flags those it could not
// complete, and those with sources that reach past its FIFO; the full-FIFO
// kernel then recomputes the incomplete tiles and the row-chunk neighbours of
// the far-reaching ones (it returns at once when nothing was flagged).  flags
// holds two ints of flag bits per tile (march2d_flag_bytes(tiles, false)
// bytes); with split, the state of the passes' row chunks follows them
// (march2d_flag_bytes(tiles, true) bytes, zero before the first step).
template <typename T>
hipError_t launch_march2d(const T* Y, T* Yn, const Grid& g, const MarchGeom& m, const Consts& k,
                          StepCtl* ctl, double* partials, int* flags, long long step, hipStream_t stream,
                          bool split);

// Row chunks of the square lattice's short and full passes: at most
// kSplitMax per tile.  Their state follows the two flag words per tile
// (flags, flags_lean): two work words per tile (written in the steps of
// each parity), one counter of finished chunks per tile (zero between
// passes), two lists of tiles to cut (written in the steps of each parity),
// the list of tiles for the full pass, then kSplitMax partial rows per tile
// (chunk p of tile t at row p * tiles + t), 8-byte aligned.  The first 5
// words per tile start at zero.
constexpr int kSplitMax = 8;
__host__ __device__ inline int64_t split_slots_offset(int64_t ntiles) { return 8 * ntiles; }
inline size_t march2d_flag_bytes(int64_t ntiles, bool split)
{
    return split ? (size_t)split_slots_offset(ntiles) * 4 + (size_t)kSplitMax * ntiles * kPartialStride * 8
                 : (size_t)2 * ntiles * 4;
}

// Hexagonal lattice (lb_hex.hip): one block per tile of 64 x 4 nodes (axial
// i x j), hex_blocks(g) blocks and partial rows per step.
template <typename T>
hipError_t launch_hex(const T* Y, T* Yn, const Grid& g, const Consts& k, StepCtl* ctl, double* partials,
                      long long step, hipStream_t stream);
int64_t hex_blocks(const Grid& g);

// Reduce nb per-block partial rows of one step into ctl (fixed order);
// species2d: also the rho chi sums of the square lattice with two gases.
hipError_t launch_finalize(double* partials, int64_t nb, StepCtl* ctl, long long step,
                           hipStream_t stream, bool species2d = false);
constexpr int kHalo = 5;

// Riemann initial state: node i (cell centre x_lo + (i + 1/2) dx) takes the
// left moments when x < x_d, else the right ones (lattice units; left and
// right hold 5 values, of which the first nf are used).
template <typename T>
hipError_t launch_init_riemann(T* Y, const Grid& g, int nf, double x_lo, double dx, double x_d,
                               const double* left, const double* right, hipStream_t stream);

// Lattice-unit state -> FP64 physical moments (divide by scale[f]; 5 values).
template <typename T>
hipError_t launch_export(const T* Y, double* out, int64_t nn, int nf, const double* scale,
                         hipStream_t stream);

// Per-node (f_x, f_y, c'_1) with the same device function as the step.
template <typename T>
hipError_t launch_lanes(const T* Y, const Grid& g, int dim, const Consts& k, int32_t* fx,
                        int32_t* fy, int32_t* c1, hipStream_t stream);

hipError_t launch_reset_ctl(StepCtl* ctl, hipStream_t stream);

// p[0 .. n) := v (a kernel, not a memset: it may be captured into a graph).
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t stream);

// *out := the outcome of the step(s) recorded in ctl: kStatusOk, or the
// status code of the first failure (the values of LB_OK, LB_ESTATE, LB_EREACH).
constexpr int kStatusOk = 0, kStatusState = -4, kStatusReach = -5;
hipError_t launch_status(const StepCtl* ctl, int32_t* out, hipStream_t stream);

// ---- pools: many independent problems advanced by one persistent launch per
// step over a device-resident tile table (lb_pool.hip) ----

struct PoolProb {       // one slot, written by the host between launches
    int64_t off[2];     // element offsets of the two SoA moment sets in the arena
    int64_t nx, ny;
    int32_t bc_x, bc_y;
    int32_t active;     // 0: free slot (it owns no tiles)
    int32_t pad;
    int64_t target;     // the problem stops after this many good steps
    int64_t t0, t1;     // its tiles [t0, t1) in the tile table
};

struct PoolState {      // one slot, written by the device, read by the host after a sync
    int64_t done;       // good steps so far: the moments are in set (done & 1)
    int64_t err_step;   // step that failed (0: none); the problem then stops
    int32_t err_code;   // kErr* bits
    int32_t max_reach;  // largest reach of its latest step
    int64_t totals_step;
    double totals[4];   // interior sums after step totals_step (lattice units)
};

struct PoolTile {        // one tile, with a copy of its slot's grid so a block reads one record
    int32_t prob, rows;  // slot; destination rows (square lattice; 1 in 1-D)
    int64_t x0, y0;      // first destination column / row
    int64_t off[2];      // the slot's two moment sets (element offsets in the arena)
    int64_t nx, ny;
    int32_t bc_x, bc_y;
};

// Per-tile word kept by the per-slot reduction: bit 0 = the set holding the
// slot's current moments (done & 1), bit 1 = the slot still steps.
constexpr int kTileSet = 1, kTileLive = 2;

struct PoolView {
    const PoolProb* probs;
    PoolState* state;
    const PoolTile* tiles;
    int32_t* tstate;        // kTileSet | kTileLive per tile
    const int32_t* ntiles;  // tiles in the table (read by the kernels, so admissions need no new launch shape)
    double* partials;       // kPartialStride doubles per tile
    int32_t* flags;         // square lattice: per-tile flag bits of the short- and full-FIFO passes
    int32_t* flags_lean;    // square lattice: per-tile flag bits of the lean pass
    int32_t* next;          // 5 counters, as StepCtl::next; reset by finalize
    void* arena;            // moment sets of all slots (T elements)
};

// Tile shapes of the 1-D pool kernel (threads per block, nodes per thread).
constexpr int kPool1Shapes = 5;
constexpr int kPool1TPB[kPool1Shapes] = {256, 256, 256, 256, 512};
constexpr int kPool1J[kPool1Shapes] = {1, 2, 4, 8, 4};
// Square-lattice pool tiles: the strip height is chosen so that the live
// problems make about kPool2TilesPerBlock[shape] tiles per resident block
// (claim-order balance against the 2L halo rows each tile marches again), and
// is at least kPool2MinRows.
constexpr int kPool2Shapes = 5;
constexpr int kPool2TilesPerBlock[kPool2Shapes] = {2, 3, 4, 6, 8};
constexpr int kPool2MinRows = 16;
constexpr int kPool2Cols = 256 - 2 * kHalo;  // destination columns per square-lattice tile

// One step of every live tile: the 1-D kernel of tile shape `shape` (nblocks =
// the number of tiles, one block each), or the square-lattice short-FIFO pass
// followed by the full-FIFO pass over the tiles it flagged (nblocks persistent
// blocks claim the tiles).
template <typename T>
hipError_t launch_pool1d(const PoolView& v, const Consts& k, int shape, int nblocks, bool walls,
                         hipStream_t stream);
template <typename T>
hipError_t launch_pool2d(const PoolView& v, const Consts& k, int nblocks_lean, int nblocks, bool walls,
                         hipStream_t stream);
// Resident blocks per CU of the pool's short pass (lean = false) or lean pass.
template <typename T>
int pool2d_blocks_per_cu(bool lean = false);
// Per slot: reduce its tiles' partial rows (fixed order) into its state and,
// when commit != 0 and the step succeeded, count the step.
hipError_t launch_pool_finalize(const PoolView& v, int nslots, int commit, hipStream_t stream);

}  // namespace lbsd
