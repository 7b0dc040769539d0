// Square-lattice pool form (many grids per launch over a tile table): the
// one-gas kernel instances (kernel templates in lb_march2d.hpp; a translation
// unit of its own so that it compiles in parallel with the plain form's).
#include "lb_march2d.hpp"

namespace lbsd {

template <typename T>
int pool2d_blocks_per_cu(bool lean)
{
    int nb = 0;
    const hipError_t e = lean
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pool2d_lean_kernel<T, false, false, false>, kMTPB, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pool2d_kernel<T, kLSmall, false, false, false>, kMTPB, 0);
    if (e != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

template <typename T>
hipError_t launch_pool2d(const PoolView& v, const Consts& k, int nblocks_lean, int nblocks, bool walls,
                         hipStream_t stream)
{
    if (k.species) return launch_pool2d_species<T>(v, k, nblocks_lean, nblocks, walls, stream);
    if (k.rest_q > 0.0)
        return walls ? launch_pool2d_w<T, true, true, false>(v, k, nblocks_lean, nblocks, stream)
                     : launch_pool2d_w<T, false, true, false>(v, k, nblocks_lean, nblocks, stream);
    return walls ? launch_pool2d_w<T, true, false, false>(v, k, nblocks_lean, nblocks, stream)
                 : launch_pool2d_w<T, false, false, false>(v, k, nblocks_lean, nblocks, stream);
}

template int pool2d_blocks_per_cu<double>(bool);
template int pool2d_blocks_per_cu<float>(bool);
template hipError_t launch_pool2d<double>(const PoolView&, const Consts&, int, int, bool, hipStream_t);
template hipError_t launch_pool2d<float>(const PoolView&, const Consts&, int, int, bool, hipStream_t);

}  // namespace lbsd
