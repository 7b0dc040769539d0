// Square-lattice step as a column march with two gases: the plain form's
// instances that carry the species moment rho chi.  The kernel templates are
// in lb_march2d.hpp; the instances are spread over translation units of their
// own (lb_march2d.hip, lb_pool2d.hip, lb_pool2d_sp.hip) that compile in
// parallel.
#include "lb_march2d.hpp"

namespace lbsd {

template <typename T>
hipError_t launch_march2d_species(const T* Y, T* Yn, const Grid& g, const MarchGeom& m, const Consts& k,
                                  StepCtl* ctl, double* partials, int* flags, long long step,
                                  hipStream_t stream, bool split)
{
    const bool walls = g.bc_x == kBcReflecting || g.bc_y == kBcReflecting, rest = k.rest_q > 0.0;
    if (rest)
        return walls ? launch_march2d_w<T, true, true, true>(Y, Yn, g, m, k, ctl, partials, flags, step, stream, split)
                     : launch_march2d_w<T, false, true, true>(Y, Yn, g, m, k, ctl, partials, flags, step, stream, split);
    return walls ? launch_march2d_w<T, true, false, true>(Y, Yn, g, m, k, ctl, partials, flags, step, stream, split)
                 : launch_march2d_w<T, false, false, true>(Y, Yn, g, m, k, ctl, partials, flags, step, stream, split);
}

template hipError_t launch_march2d_species<double>(const double*, double*, const Grid&, const MarchGeom&,
                                                   const Consts&, StepCtl*, double*, int*, long long,
                                                   hipStream_t, bool);
template hipError_t launch_march2d_species<float>(const float*, float*, const Grid&, const MarchGeom&,
                                                  const Consts&, StepCtl*, double*, int*, long long,
                                                  hipStream_t, bool);

}  // namespace lbsd
