// Square-lattice step as a column march with two gases: the instances (plain
// and pool form) that carry the species moment rho chi.  The kernel templates
// are in lb_march2d.hpp; this translation unit of its own lets the one-gas and
// two-gas halves compile in parallel.
#include "lb_march2d.hpp"

namespace lbsd {

template <typename T>
hipError_t launch_march2d_species(const T* Y, T* Yn, const Grid& g, const MarchGeom& m, const Consts& k,
                                  StepCtl* ctl, double* partials, int* flags, long long step,
                                  hipStream_t stream)
{
    const bool walls = g.bc_x == kBcReflecting || g.bc_y == kBcReflecting, rest = k.rest_q > 0.0;
    if (rest)
        return walls ? launch_march2d_w<T, true, true, true>(Y, Yn, g, m, k, ctl, partials, flags, step, stream)
                     : launch_march2d_w<T, false, true, true>(Y, Yn, g, m, k, ctl, partials, flags, step, stream);
    return walls ? launch_march2d_w<T, true, false, true>(Y, Yn, g, m, k, ctl, partials, flags, step, stream)
                 : launch_march2d_w<T, false, false, true>(Y, Yn, g, m, k, ctl, partials, flags, step, stream);
}

template <typename T>
hipError_t launch_pool2d_species(const PoolView& v, const Consts& k, int nblocks, bool walls, hipStream_t stream)
{
    if (k.rest_q > 0.0)
        return walls ? launch_pool2d_w<T, true, true, true>(v, k, nblocks, stream)
                     : launch_pool2d_w<T, false, true, true>(v, k, nblocks, stream);
    return walls ? launch_pool2d_w<T, true, false, true>(v, k, nblocks, stream)
                 : launch_pool2d_w<T, false, false, true>(v, k, nblocks, stream);
}

template hipError_t launch_march2d_species<double>(const double*, double*, const Grid&, const MarchGeom&,
                                                   const Consts&, StepCtl*, double*, int*, long long,
                                                   hipStream_t);
template hipError_t launch_march2d_species<float>(const float*, float*, const Grid&, const MarchGeom&,
                                                  const Consts&, StepCtl*, double*, int*, long long,
                                                  hipStream_t);

template hipError_t launch_pool2d_species<double>(const PoolView&, const Consts&, int, bool, hipStream_t);
template hipError_t launch_pool2d_species<float>(const PoolView&, const Consts&, int, bool, hipStream_t);

}  // namespace lbsd
