// Host-side helpers shared by the solver (lb_api.hip) and the pool
// (lb_pool.hip) runtimes.
#pragma once
#include "lb_kernels.hpp"
#include "lbsd.h"

namespace lbsd {

// Record a message for lb_last_error() and return `code`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_fail(hipError_t e, const char* what);
size_t align256(size_t n);

// Argument checks shared by lb_create and the pool calls (LB_OK or LB_EINVAL).
int check_model(int dim, double gamma, const lb_velset* vs, int precision);
int check_grid(const lb_grid* grid, int dim);
Consts make_consts(int dim, double gamma, const lb_velset* vs);
bool is_hex(const lb_velset* vs);  // one of the hexagonal sets

// Riemann states in lattice units: lambda = lam_set if > 0, else cfl over
// the largest |u| + sqrt(gamma p / rho) of the two states; side[i] holds
// rho, rho u lambda, (rho v lambda), rho E lambda^2 (eq. 27 for rho E) and,
// with two gases (species), rho chi: gas 1 (gamma_l) on the left, gas 2
// (gamma_r) on the right.  side[i][4] is 0 where nf < 5.
int riemann_sides(int dim, double gamma_l, double gamma_r, bool species, double lam_set, double cfl,
                  const lb_prim* L, const lb_prim* R, double* lam_out, double side[2][5]);
// rho > 0 and finite everywhere (LB_ESTATE otherwise).
int check_moments(const double* Y, int nf, int64_t nn);
// Two gases: the last field, rho chi, within [0, rho] (LB_ESTATE otherwise).
int check_species(const double* Y, int nf, int64_t nn);
// Physical FP64 SoA moments -> lattice units of the storage type, copied to
// dst on `stream` (synchronously).  ie: index of the rho E field.
int upload_moments(void* dst, const double* Y, int nf, int ie, int64_t nn, double lambda, bool fp64,
                   hipStream_t stream);
// Lattice -> physical divisor per field: 1 (rho, rho chi), lambda (momenta),
// lambda^2 (rho E, field ie).
void field_scales(int nf, int ie, double lambda, double sc[5]);

}  // namespace lbsd
