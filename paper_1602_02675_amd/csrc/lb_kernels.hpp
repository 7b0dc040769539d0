// Kernel-side interface shared by the step kernels and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lb_device.hpp"

namespace lbsd {

constexpr int kBcTransmissive = 0;
constexpr int kBcPeriodic = 1;

constexpr int kErrReach = 1;  // a packet would travel further than the halo
constexpr int kErrState = 2;  // rho <= 0 or a non-finite moment

// Per-solver control block in device memory (written by the step kernels).
struct StepCtl {
    unsigned int counter;   // blocks of the running step that are done
    int err_code;           // kErr* bits of the first failed step
    long long err_step;     // first failed step (LLONG_MAX if none)
    long long totals_step;  // step whose totals are in `totals`
    double totals[4];       // interior sums of the moment fields (lattice units)
    int max_reach;          // largest reach seen in the latest step
    int pad[7];
};

// Per-block partial results: 4 field sums, reach, error bits.
constexpr int kPartialStride = 8;

struct Grid {
    int64_t nx, ny;  // ny = 1 in 1-D
    int bc_x, bc_y;
};

// Launch one step of a 1-D / 2-D problem (async on `stream`).  Y and Yn are
// SoA [nf][ny][nx] arrays of T; partials holds one kPartialStride row per
// block (step_blocks_* gives the count).
template <typename T>
hipError_t launch_step1d(const T* Y, T* Yn, const Grid& g, const Consts& k, StepCtl* ctl,
                         double* partials, long long step, hipStream_t stream);
template <typename T>
hipError_t launch_step2d(const T* Y, T* Yn, const Grid& g, const Consts& k, StepCtl* ctl,
                         double* partials, long long step, hipStream_t stream);
int64_t step_blocks_1d(const Grid& g);
int64_t step_blocks_2d(const Grid& g);
constexpr int kHalo = 5;

// Riemann initial state: node i (cell centre x_lo + (i + 1/2) dx) takes the
// left moments when x < x_d, else the right ones (lattice units).
template <typename T>
hipError_t launch_init_riemann(T* Y, const Grid& g, int nf, double x_lo, double dx, double x_d,
                               const double* left, const double* right, hipStream_t stream);

// Lattice-unit state -> FP64 physical moments (divide by scale[f]).
template <typename T>
hipError_t launch_export(const T* Y, double* out, int64_t nn, int nf, const double* scale,
                         hipStream_t stream);

// Per-node (f_x, f_y, c'_1) with the same device function as the step.
template <typename T>
hipError_t launch_lanes(const T* Y, const Grid& g, int dim, const Consts& k, int32_t* fx,
                        int32_t* fy, int32_t* c1, hipStream_t stream);

hipError_t launch_reset_ctl(StepCtl* ctl, hipStream_t stream);

}  // namespace lbsd
