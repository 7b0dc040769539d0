// Square-lattice pool form with two gases: the pool kernels' instances that
// carry the species moment rho chi (kernel templates in lb_march2d.hpp; a
// translation unit of its own so that it compiles in parallel).
#include "lb_march2d.hpp"

namespace lbsd {

template <typename T>
hipError_t launch_pool2d_species(const PoolView& v, const Consts& k, int nblocks_lean, int nblocks, bool walls,
                                 hipStream_t stream)
{
    if (k.rest_q > 0.0)
        return walls ? launch_pool2d_w<T, true, true, true>(v, k, nblocks_lean, nblocks, stream)
                     : launch_pool2d_w<T, false, true, true>(v, k, nblocks_lean, nblocks, stream);
    return walls ? launch_pool2d_w<T, true, false, true>(v, k, nblocks_lean, nblocks, stream)
                 : launch_pool2d_w<T, false, false, true>(v, k, nblocks_lean, nblocks, stream);
}

template hipError_t launch_pool2d_species<double>(const PoolView&, const Consts&, int, int, bool, hipStream_t);
template hipError_t launch_pool2d_species<float>(const PoolView&, const Consts&, int, int, bool, hipStream_t);

}  // namespace lbsd
