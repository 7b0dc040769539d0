// Small kernels around the step: Riemann initial state, moment export,
// per-node lane dump and control-block reset.
#include <climits>

#include "lb_kernels.hpp"

namespace lbsd {

namespace {

template <typename T>
__global__ void init_riemann_kernel(T* __restrict__ Y, int64_t nx, int64_t nn, int nf, double x_lo,
                                    double dx, double x_d, double l0, double l1, double l2, double l3,
                                    double l4, double r0, double r1, double r2, double r3, double r4)
{
#pragma clang fp contract(off)
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nn) return;
    const int64_t i = q % nx;
    const double x = x_lo + ((double)i + 0.5) * dx;  // cell centre
    const bool left = x < x_d;
    const double v[5] = {left ? l0 : r0, left ? l1 : r1, left ? l2 : r2, left ? l3 : r3, left ? l4 : r4};
    for (int f = 0; f < nf; ++f) Y[(int64_t)f * nn + q] = (T)v[f];
}

template <typename T>
__global__ void export_kernel(const T* __restrict__ Y, double* __restrict__ out, int64_t nn, int nf,
                              double s0, double s1, double s2, double s3, double s4)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nn) return;
    const double s[5] = {s0, s1, s2, s3, s4};
    for (int f = 0; f < nf; ++f) out[(int64_t)f * nn + q] = (double)Y[(int64_t)f * nn + q] / s[f];
}

template <typename T>
__global__ void lanes_kernel(const T* __restrict__ Y, int64_t nn, int dim, Consts k,
                             int32_t* __restrict__ fx, int32_t* __restrict__ fy,
                             int32_t* __restrict__ c1)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nn) return;
    if (dim == 1) {
        // the same device function the step uses (one gas, or the mixture of two)
        const Src1<T> s = k.species ? make_src1<T, true>(Y[q], Y[nn + q], Y[2 * nn + q], k, Y[3 * nn + q])
                                    : make_src1<T, false>(Y[q], Y[nn + q], Y[2 * nn + q], k);
        fx[q] = s.f;
        fy[q] = 0;
        c1[q] = s.c1;
    } else if (k.hex) {
        // hexagonal lattice: the floors of the axial coordinates of v
        const T m0 = Y[q], m1 = Y[nn + q], m2 = Y[2 * nn + q], m3 = Y[3 * nn + q];
        const SrcHex<T> s = k.b0 > 0.0 ? make_srchex<T, true>(m0, m1, m2, m3, k)
                                       : make_srchex<T, false>(m0, m1, m2, m3, k);
        fx[q] = s.fa;
        fy[q] = s.fb;
        c1[q] = s.c1;
    } else {
        // the same device function the step uses (with or without the rest group)
        const T m0 = Y[q], m1 = Y[nn + q], m2 = Y[2 * nn + q], m3 = Y[3 * nn + q];
        const bool rest = k.rest_q > 0.0;
        const Src2<T> s = k.species ? (rest ? make_src2<T, true, true>(m0, m1, m2, m3, k, Y[4 * nn + q])
                                            : make_src2<T, false, true>(m0, m1, m2, m3, k, Y[4 * nn + q]))
                                    : (rest ? make_src2<T, true>(m0, m1, m2, m3, k)
                                            : make_src2<T, false>(m0, m1, m2, m3, k));
        fx[q] = s.fx;
        fy[q] = s.fy;
        c1[q] = s.c1;
    }
}

__global__ void reset_ctl_kernel(StepCtl* ctl)
{
    if (threadIdx.x == 0) {
        for (int i = 0; i < 5; ++i) ctl->next[i] = 0;
        ctl->err_code = 0;
        ctl->err_step = LLONG_MAX;
        ctl->totals_step = -1;
        for (int f = 0; f < 4; ++f) ctl->totals[f] = 0.0;
        ctl->totals_sp = 0.0;
        ctl->max_reach = 0;
        ctl->redo_tiles = 0;
        ctl->keep[0] = 0;
        ctl->keep[1] = 0;
        ctl->split_n[0] = 0;
        ctl->split_n[1] = 0;
        ctl->full_n = 0;
    }
}

// The step's outcome as an lbsd status code (LB_OK, LB_EREACH, LB_ESTATE).
__global__ void status_kernel(const StepCtl* __restrict__ ctl, int32_t* __restrict__ out)
{
    if (threadIdx.x == 0) {
        const int e = ctl->err_code;
        *out = e == 0 ? 0 : ((e & kErrState) ? kStatusState : kStatusReach);
    }
}

__global__ void fill_i32_kernel(int32_t* __restrict__ p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

unsigned blocks_for(int64_t n, int tpb) { return (unsigned)((n + tpb - 1) / tpb); }

}  // namespace

template <typename T>
hipError_t launch_init_riemann(T* Y, const Grid& g, int nf, double x_lo, double dx, double x_d,
                               const double* l, const double* r, hipStream_t stream)
{
    const int64_t nn = g.nx * g.ny;
    init_riemann_kernel<T><<<blocks_for(nn, 256), 256, 0, stream>>>(
        Y, g.nx, nn, nf, x_lo, dx, x_d, l[0], l[1], l[2], l[3], l[4], r[0], r[1], r[2], r[3], r[4]);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_export(const T* Y, double* out, int64_t nn, int nf, const double* s,
                         hipStream_t stream)
{
    export_kernel<T><<<blocks_for(nn, 256), 256, 0, stream>>>(Y, out, nn, nf, s[0], s[1], s[2], s[3], s[4]);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_lanes(const T* Y, const Grid& g, int dim, const Consts& k, int32_t* fx,
                        int32_t* fy, int32_t* c1, hipStream_t stream)
{
    const int64_t nn = g.nx * g.ny;
    lanes_kernel<T><<<blocks_for(nn, 256), 256, 0, stream>>>(Y, nn, dim, k, fx, fy, c1);
    return hipGetLastError();
}

hipError_t launch_reset_ctl(StepCtl* ctl, hipStream_t stream)
{
    reset_ctl_kernel<<<1, 64, 0, stream>>>(ctl);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    fill_i32_kernel<<<blocks_for(n, 256), 256, 0, stream>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_status(const StepCtl* ctl, int32_t* out, hipStream_t stream)
{
    status_kernel<<<1, 64, 0, stream>>>(ctl, out);
    return hipGetLastError();
}

template hipError_t launch_init_riemann<double>(double*, const Grid&, int, double, double, double,
                                                const double*, const double*, hipStream_t);
template hipError_t launch_init_riemann<float>(float*, const Grid&, int, double, double, double,
                                               const double*, const double*, hipStream_t);
template hipError_t launch_export<double>(const double*, double*, int64_t, int, const double*,
                                          hipStream_t);
template hipError_t launch_export<float>(const float*, double*, int64_t, int, const double*,
                                         hipStream_t);
template hipError_t launch_lanes<double>(const double*, const Grid&, int, const Consts&, int32_t*,
                                         int32_t*, int32_t*, hipStream_t);
template hipError_t launch_lanes<float>(const float*, const Grid&, int, const Consts&, int32_t*,
                                        int32_t*, int32_t*, hipStream_t);

}  // namespace lbsd
