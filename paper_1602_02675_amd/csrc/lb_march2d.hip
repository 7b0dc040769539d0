// Square-lattice step as a column march: the one-gas instances of the plain
// form and the launch geometry (the kernel templates and how the march works
// are in lb_march2d.hpp; the pool form's one-gas instances are in
// lb_pool2d.hip, the two-gas instances in lb_march2d_sp.hip and
// lb_pool2d_sp.hip).
#include <algorithm>

#include "lb_march2d.hpp"

namespace lbsd {

namespace {

int64_t x_strips(const Grid& g) { return (g.nx + (kMTPB - 2 * kMH) - 1) / (kMTPB - 2 * kMH); }

}  // namespace

#ifndef LB_MARCH_TILES_X10
#define LB_MARCH_TILES_X10 10  // tiles per resident block of the lean pass, times 10
#endif
MarchGeom march2d_geometry(const Grid& g, int cus, int per_cu, int per_cu_lean)
{
    MarchGeom m;
    const int64_t xs = x_strips(g);
    const int64_t resident = (int64_t)(cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
    const int64_t resident_lean = (int64_t)(cus > 0 ? cus : 1) * (per_cu_lean > 0 ? per_cu_lean : 1);
    // a whole number of tiles per resident block of both the lean pass, which
    // does the bulk of a planar step, and the short pass, which does it where
    // the flow is not planar: the least common multiple of the two block
    // counts when that is at most twice the larger, else about
    // LB_MARCH_TILES_X10 / 10 tiles per lean block (its tiles cost about the
    // same; taller tiles march fewer halo rows again); strips no shorter than
    // kMinRows.  Rounded down: one tile more than a multiple of the resident
    // blocks would cost a pass a second round for that tile.
    int64_t a = resident_lean, b = resident;
    while (b != 0) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    const int64_t lcm = resident_lean / a * resident;
    const int64_t want = lcm <= 2 * std::max(resident, resident_lean)
                             ? lcm
                             : (int64_t)LB_MARCH_TILES_X10 * resident_lean / 10;
    int64_t chunks = want / xs;
    if (chunks < 1) chunks = 1;
    int64_t sy = (g.ny + chunks - 1) / chunks;
    if (sy < kMinRows) sy = kMinRows;
    m.sy = (int)sy;
    m.grid_x = xs;
    m.grid_y = (g.ny + sy - 1) / sy;
    m.nblocks = (int)std::min<int64_t>(resident, m.blocks());
    m.nblocks_lean = (int)std::min<int64_t>(resident_lean, m.blocks());
    return m;
}

int64_t march2d_max_blocks(const Grid& g)
{
    return x_strips(g) * ((g.ny + kMinRows - 1) / kMinRows);
}

template <typename T>
int march2d_blocks_per_cu(bool lean)
{
    int nb = 0;
    const hipError_t e = lean
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, march2d_lean_kernel<T, false, false, false>, kMTPB, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, march2d_kernel<T, kLSmall, false, false, false>, kMTPB, 0);
    if (e != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

// Grids without reflecting walls run the instances that keep no mirror state,
// the dual-level set those without the rest group.
template <typename T>
hipError_t launch_march2d(const T* Y, T* Yn, const Grid& g, const MarchGeom& m, const Consts& k,
                          StepCtl* ctl, double* partials, int* flags, long long step, hipStream_t stream,
                          bool split)
{
    const bool walls = g.bc_x == kBcReflecting || g.bc_y == kBcReflecting, rest = k.rest_q > 0.0;
    if (k.species) return launch_march2d_species<T>(Y, Yn, g, m, k, ctl, partials, flags, step, stream, split);
    if (rest)
        return walls ? launch_march2d_w<T, true, true, false>(Y, Yn, g, m, k, ctl, partials, flags, step, stream, split)
                     : launch_march2d_w<T, false, true, false>(Y, Yn, g, m, k, ctl, partials, flags, step, stream, split);
    return walls ? launch_march2d_w<T, true, false, false>(Y, Yn, g, m, k, ctl, partials, flags, step, stream, split)
                 : launch_march2d_w<T, false, false, false>(Y, Yn, g, m, k, ctl, partials, flags, step, stream, split);
}

template int march2d_blocks_per_cu<double>(bool);
template int march2d_blocks_per_cu<float>(bool);
template hipError_t launch_march2d<double>(const double*, double*, const Grid&, const MarchGeom&,
                                           const Consts&, StepCtl*, double*, int*, long long, hipStream_t, bool);
template hipError_t launch_march2d<float>(const float*, float*, const Grid&, const MarchGeom&,
                                          const Consts&, StepCtl*, double*, int*, long long, hipStream_t, bool);

}  // namespace lbsd
