// Host runtime behind include/lbsd.h: validation, device-memory layout
// inside the caller's buffer, launches on the caller's stream, error
// recovery to the last good step.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <climits>
#include <mutex>
#include <string>
#include <vector>

#include "lb_host.hpp"

using namespace lbsd;

namespace lbsd {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(LB_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

int check_model(int dim, double gamma, const lb_velset* vs, int precision)
{
    if (!vs) return fail(LB_EINVAL, "null velocity set");
    if (dim != 1 && dim != 2) return fail(LB_EINVAL, "dim must be 1 or 2 (got %d)", dim);
    if (!(gamma > 1.0) || !(gamma <= 1.0 + 2.0 / dim))
        return fail(LB_EINVAL, "gamma must lie in (1, 1 + 2/D] (phi >= 0, eq. 15); got %g", gamma);
    if ((dim == 1 && vs->lattice != LB_LATTICE_D1_TRIPLE) ||
        (dim == 2 && vs->lattice != LB_LATTICE_D2_SQUARE_DUAL && vs->lattice != LB_LATTICE_D2_SQUARE_TRIPLE &&
         vs->lattice != LB_LATTICE_D2_HEX_DUAL && vs->lattice != LB_LATTICE_D2_HEX_TRIPLE))
        return fail(LB_EINVAL, "lattice %d does not match dim %d", vs->lattice, dim);
    if (vs->lattice == LB_LATTICE_D2_HEX_DUAL && vs->d0_frac != 0.0)
        return fail(LB_EINVAL, "the hexagonal dual-level set has d0 = 0");
    if (vs->lattice == LB_LATTICE_D2_HEX_TRIPLE && !(vs->d0_frac > 0.0 && vs->d0_frac < 1.0))
        return fail(LB_EINVAL, "the hexagonal set with a rest group needs d0_frac in (0, 1); got %g", vs->d0_frac);
    if (dim == 1 && !(vs->d0_frac >= 0.0 && vs->d0_frac < 1.0))
        return fail(LB_EINVAL, "d0_frac must lie in [0, 1); got %g", vs->d0_frac);
    if (vs->lattice == LB_LATTICE_D2_SQUARE_DUAL && vs->d0_frac != 0.0)
        return fail(LB_EINVAL, "the square dual-level set has d0 = 0");
    if (vs->lattice == LB_LATTICE_D2_SQUARE_TRIPLE && !(vs->d0_frac > 0.0 && vs->d0_frac < 1.0))
        return fail(LB_EINVAL, "the square set with a rest level needs d0_frac in (0, 1); got %g", vs->d0_frac);
    if (precision != LB_FP64 && precision != LB_FP32)
        return fail(LB_EINVAL, "precision must be LB_FP64 or LB_FP32");
    return LB_OK;
}

int check_grid(const lb_grid* grid, int dim)
{
    if (!grid) return fail(LB_EINVAL, "null grid");
    if (grid->dim != dim) return fail(LB_EINVAL, "grid dim %d, expected %d", grid->dim, dim);
    if (grid->nx < 1 || grid->ny < 1) return fail(LB_EINVAL, "nx, ny must be >= 1");
    if (dim == 1 && grid->ny != 1) return fail(LB_EINVAL, "ny must be 1 in 1-D");
    if (grid->nx > (int64_t)1 << 40 || grid->ny > (int64_t)1 << 40 ||
        grid->nx * grid->ny > (int64_t)1 << 36)
        return fail(LB_EINVAL, "grid too large");
    // the square-lattice kernels address a row's nodes with 32-bit byte offsets
    if (dim == 2 && grid->nx > (int64_t)1 << 28) return fail(LB_EINVAL, "nx must be <= 2^28 on the 2-D lattices");
    if (!(grid->x_hi > grid->x_lo) || !isfinite(grid->x_lo) || !isfinite(grid->x_hi))
        return fail(LB_EINVAL, "need x_lo < x_hi");
    for (int b : {grid->bc_x, grid->bc_y})
        if (b != LB_BC_TRANSMISSIVE && b != LB_BC_PERIODIC && b != LB_BC_REFLECTING)
            return fail(LB_EINVAL, "unknown boundary condition %d", b);
    // mirror images of the halo nodes must lie inside the grid
    if (grid->bc_x == LB_BC_REFLECTING && grid->nx < LB_HALO)
        return fail(LB_EINVAL, "reflecting walls along x need nx >= %d", LB_HALO);
    if (dim == 2 && grid->bc_y == LB_BC_REFLECTING && grid->ny < LB_HALO)
        return fail(LB_EINVAL, "reflecting walls along y need ny >= %d", LB_HALO);
    return LB_OK;
}

bool is_hex(const lb_velset* vs)
{
    return vs->lattice == LB_LATTICE_D2_HEX_DUAL || vs->lattice == LB_LATTICE_D2_HEX_TRIPLE;
}

Consts make_consts(int dim, double gamma, const lb_velset* vs)
{
    Consts k;
    k.Dg1 = (double)dim * (gamma - 1.0);
    k.phi_coef = 1.0 - ((double)dim / 2.0) * (gamma - 1.0);
    k.hex = is_hex(vs) ? 1 : 0;
    const bool rest = dim == 1 || vs->lattice == LB_LATTICE_D2_SQUARE_TRIPLE || vs->lattice == LB_LATTICE_D2_HEX_TRIPLE;
    k.delta0 = rest ? vs->d0_frac : 0.0;
    k.b0 = rest ? 1.0 : 0.0;
    k.inv_b1 = dim == 1 ? 0.5 : (k.hex ? 1.0 / 6.0 : 0.25);
    // square lattice with a rest level: d_0 = q (d_1 + d_2), q = b_1 delta0 / (1 - delta0),
    // so that a rest packet's mass follows from the staged level masses
    k.rest_q = (dim == 2 && rest && !k.hex) ? 4.0 * vs->d0_frac / (1.0 - vs->d0_frac) : 0.0;
    return k;
}

static bool prim_ok(const lb_prim* p)
{
    return p && p->rho > 0.0 && p->p >= 0.0 && isfinite(p->rho) && isfinite(p->u) &&
           isfinite(p->v) && isfinite(p->p);
}

int riemann_sides(int dim, double gamma_l, double gamma_r, bool species, double lam_set, double cfl,
                  const lb_prim* L, const lb_prim* R, double* lam_out, double side[2][5])
{
    if (!prim_ok(L) || !prim_ok(R)) return fail(LB_ESTATE, "need rho > 0, p >= 0, finite values");
    const double gs[2] = {gamma_l, gamma_r};
    double lam = lam_set;
    if (!(lam > 0.0)) {
        double smax = 0.0;
        for (int i = 0; i < 2; ++i) {
            const lb_prim* q = i == 0 ? L : R;
            const double uu = dim == 2 ? sqrt(q->u * q->u + q->v * q->v) : fabs(q->u);
            const double c = uu + sqrt(gs[i] * q->p / q->rho);
            smax = c > smax ? c : smax;
        }
        if (!(smax > 0.0)) return fail(LB_ESTATE, "both states have zero signal speed; set lambda");
        lam = cfl / smax;
    }
    const lb_prim* P[2] = {L, R};
    const double lam2 = lam * lam;
    for (int i = 0; i < 2; ++i) {
        const double rho = P[i]->rho, u = P[i]->u, v = dim == 2 ? P[i]->v : 0.0, p = P[i]->p;
        const double rE = p / (gs[i] - 1.0) + 0.5 * rho * (u * u + v * v);
        side[i][0] = rho;
        side[i][1] = (rho * u) * lam;
        side[i][4] = 0.0;
        if (dim == 2) {
            side[i][2] = (rho * v) * lam;
            side[i][3] = rE * lam2;
            side[i][4] = species && i == 0 ? rho : 0.0;  // gas 1 fills the left side
        } else {
            side[i][2] = rE * lam2;
            side[i][3] = species && i == 0 ? rho : 0.0;
        }
    }
    *lam_out = lam;
    return LB_OK;
}

int check_moments(const double* Y, int nf, int64_t nn)
{
    if (!Y) return fail(LB_EINVAL, "null moments");
    for (int64_t q = 0; q < nn; ++q)
        if (!(Y[q] > 0.0)) return fail(LB_ESTATE, "rho <= 0 at node %lld", (long long)q);
    for (int64_t q = 0; q < (int64_t)nf * nn; ++q)
        if (!isfinite(Y[q])) return fail(LB_ESTATE, "non-finite moment at %lld", (long long)q);
    return LB_OK;
}

int check_species(const double* Y, int nf, int64_t nn)
{
    const double* chi = Y + (size_t)(nf - 1) * nn;  // the mass of gas 1 lies in [0, rho]
    for (int64_t q = 0; q < nn; ++q)
        if (!(chi[q] >= 0.0 && chi[q] <= Y[q] * (1.0 + 1e-12)))
            return fail(LB_ESTATE, "rho chi outside [0, rho] at node %lld", (long long)q);
    return LB_OK;
}

int upload_moments(void* dst, const double* Y, int nf, int ie, int64_t nn, double lambda, bool fp64,
                   hipStream_t stream)
{
    const double lam2 = lambda * lambda;
    std::vector<double> tmp;
    std::vector<float> tmpf;
    try {
        if (fp64) tmp.resize((size_t)nf * nn);
        else tmpf.resize((size_t)nf * nn);
    } catch (...) {
        return fail(LB_ENOMEM, "host staging allocation failed");
    }
    for (int f = 0; f < nf; ++f) {
        const double sc = f == ie ? lam2 : lambda;
        for (int64_t q = 0; q < nn; ++q) {
            const double y = Y[(int64_t)f * nn + q];
            const double v = (f == 0 || f > ie) ? y : y * sc;
            if (fp64) tmp[(size_t)f * nn + q] = v;
            else tmpf[(size_t)f * nn + q] = (float)v;
        }
    }
    hipError_t e = fp64 ? hipMemcpyAsync(dst, tmp.data(), tmp.size() * 8, hipMemcpyHostToDevice, stream)
                        : hipMemcpyAsync(dst, tmpf.data(), tmpf.size() * 4, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "sync");
    return LB_OK;
}

void field_scales(int nf, int ie, double lambda, double sc[5])
{
    const double lam2 = lambda * lambda;
    for (int f = 0; f < 5; ++f) sc[f] = 1.0;
    for (int f = 1; f < ie && f < nf; ++f) sc[f] = lambda;
    if (ie < nf) sc[ie] = lam2;
}

}  // namespace lbsd

struct lb_solver {
    lb_grid grid;
    Grid g;
    int dim, nf, precision;
    double gamma, gamma2;  // gamma2: gas 2 (two gases), else gamma
    bool species;          // two gases: a species field rho chi after rho E
    bool hex;              // the hexagonal lattice
    lb_velset vs;
    Consts k;
    int64_t nn;
    size_t elem;
    // layout inside the bound buffer
    size_t off_buf[2], off_export, off_ctl, off_partials, off_flags, total;
    int64_t nblocks;      // step-kernel blocks (rows of partials used per step)
    MarchGeom march;      // square lattice launch geometry (set at bind)
    char* base;
    hipStream_t stream;
    bool bound, initialized;
    double lambda_set, cfl, lambda;
    int cur;               // buffer holding the state after `steps_done` steps
    int64_t steps_done;    // steps queued since init (optimistic until synced)
    int pending_err;       // error already known on the host
    hipEvent_t ev0, ev1;
    bool events;
};

static void* buf_ptr(lb_solver* s, int i) { return s->base + s->off_buf[i]; }
static StepCtl* ctl_ptr(lb_solver* s) { return (StepCtl*)(s->base + s->off_ctl); }
static double* partials_ptr(lb_solver* s) { return (double*)(s->base + s->off_partials); }
static int* flags_ptr(lb_solver* s) { return (int*)(s->base + s->off_flags); }
static double* export_ptr(lb_solver* s) { return (double*)(s->base + s->off_export); }

extern "C" {

const char* lb_last_error(void) { return g_last_error.c_str(); }

static int create_solver(const lb_grid* grid, double gamma, double gamma2, bool species, const lb_velset* vs,
                         int32_t precision, lb_solver** out)
{
    if (!grid || !vs || !out) return fail(LB_EINVAL, "null argument");
    const int dim = grid->dim;
    int rc = check_model(dim, gamma, vs, precision);
    if (rc != LB_OK) return rc;
    if (species) {
        if ((rc = check_model(dim, gamma2, vs, precision)) != LB_OK) return rc;
    }
    if ((rc = check_grid(grid, dim)) != LB_OK) return rc;
    const bool hex = is_hex(vs);
    if (hex && species) return fail(LB_EINVAL, "the hexagonal lattice runs one gas");
    if (hex && (grid->bc_x == LB_BC_REFLECTING || grid->bc_y == LB_BC_REFLECTING))
        return fail(LB_EINVAL, "the hexagonal lattice has transmissive or periodic boundaries");

    lb_solver* s = new (std::nothrow) lb_solver();
    if (!s) return fail(LB_ENOMEM, "host allocation failed");
    s->grid = *grid;
    s->g = Grid{grid->nx, grid->ny, grid->bc_x, grid->bc_y};
    s->dim = dim;
    s->species = species;
    s->nf = dim + 2 + (species ? 1 : 0);
    s->precision = precision;
    s->gamma = gamma;
    s->gamma2 = species ? gamma2 : gamma;
    s->vs = *vs;
    s->k = make_consts(dim, gamma, vs);
    s->k.g1m1 = gamma - 1.0;
    s->k.g2m1 = s->gamma2 - 1.0;
    s->k.species = species ? 1 : 0;
    s->nn = grid->nx * grid->ny;
    s->elem = precision == LB_FP64 ? 8 : 4;
    const size_t field_bytes = align256((size_t)s->nf * (size_t)s->nn * s->elem);
    s->hex = hex;
    s->nblocks = dim == 1 ? step_blocks_1d(s->g) : (hex ? hex_blocks(s->g) : march2d_max_blocks(s->g));
    s->off_buf[0] = 0;
    s->off_buf[1] = field_bytes;
    s->off_export = 2 * field_bytes;
    s->off_ctl = s->off_export + align256((size_t)s->nf * (size_t)s->nn * 8);
    s->off_partials = s->off_ctl + align256(sizeof(StepCtl));
    s->off_flags = s->off_partials + align256((size_t)s->nblocks * kPartialStride * 8);
    // square lattice: two flag words per tile (short and full passes, lean
    // pass) and the state of the passes' row chunks; hexagonal: unused
    const size_t flag_bytes = dim == 2 ? (hex ? (size_t)2 * s->nblocks * 4 : march2d_flag_bytes(s->nblocks, true)) : 4;
    s->total = s->off_flags + align256(flag_bytes);
    s->cfl = 1.0;
    s->lambda_set = 0.0;
    *out = s;
    return LB_OK;
}

int lb_create(const lb_grid* grid, double gamma, const lb_velset* vs, int32_t precision,
              lb_solver** out)
{
    return create_solver(grid, gamma, gamma, false, vs, precision, out);
}

int lb_create_two_gas(const lb_grid* grid, double gamma_1, double gamma_2, const lb_velset* vs,
                      int32_t precision, lb_solver** out)
{
    return create_solver(grid, gamma_1, gamma_2, true, vs, precision, out);
}

size_t lb_state_bytes(const lb_solver* s) { return s ? s->total : 0; }

int lb_bind(lb_solver* s, void* dev_ptr, size_t bytes, void* hip_stream)
{
    if (!s || !dev_ptr) return fail(LB_EINVAL, "null argument");
    if (bytes < s->total) return fail(LB_ENOMEM, "buffer of %zu bytes < %zu needed", bytes, s->total);
    if ((uintptr_t)dev_ptr % 256 != 0) return fail(LB_EINVAL, "device buffer must be 256-byte aligned");
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, dev_ptr);
    if (e != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return fail(LB_EINVAL, "pointer is not device memory");
    }
    s->base = (char*)dev_ptr;
    s->stream = (hipStream_t)hip_stream;
    if (!s->events) {
        if ((e = hipEventCreate(&s->ev0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
        if ((e = hipEventCreate(&s->ev1)) != hipSuccess) return hip_fail(e, "hipEventCreate");
        s->events = true;
    }
    if (s->dim == 2 && !s->hex) {
        int dev = 0, cus = 0;
        if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
            return hip_fail(e, "hipDeviceGetAttribute");
        const bool fp64 = s->precision == LB_FP64;
        const int per_cu = fp64 ? march2d_blocks_per_cu<double>(false) : march2d_blocks_per_cu<float>(false);
        const int per_cu_lean = fp64 ? march2d_blocks_per_cu<double>(true) : march2d_blocks_per_cu<float>(true);
        s->march = march2d_geometry(s->g, cus, per_cu, per_cu_lean);
        s->nblocks = s->march.blocks();
    }
    s->bound = true;
    s->initialized = false;
    if ((e = launch_reset_ctl(ctl_ptr(s), s->stream)) != hipSuccess) return hip_fail(e, "reset");
    return LB_OK;
}

int lb_set_lambda(lb_solver* s, double lambda)
{
    if (!s || !(lambda > 0.0) || !isfinite(lambda)) return fail(LB_EINVAL, "lambda must be > 0");
    s->lambda_set = lambda;
    return LB_OK;
}

int lb_set_cfl(lb_solver* s, double cfl)
{
    if (!s || !(cfl > 0.0) || !isfinite(cfl)) return fail(LB_EINVAL, "cfl must be > 0");
    s->cfl = cfl;
    s->lambda_set = 0.0;
    return LB_OK;
}

static int start_state(lb_solver* s)
{
    s->cur = 0;
    s->steps_done = 0;
    s->pending_err = 0;
    s->initialized = true;
    hipError_t e = launch_reset_ctl(ctl_ptr(s), s->stream);
    // square lattice: the passes' per-tile flag words, work words and chunk
    // counters start clear
    if (e == hipSuccess && s->dim == 2)
        e = launch_fill_i32(flags_ptr(s), (s->hex ? 2 : 5) * s->nblocks, 0, s->stream);
    return e == hipSuccess ? LB_OK : hip_fail(e, "reset");
}

int lb_init_riemann(lb_solver* s, double x_d, const lb_prim* L, const lb_prim* R)
{
    if (!s || !s->bound) return fail(LB_EINVAL, "solver not bound");
    if (!isfinite(x_d)) return fail(LB_EINVAL, "diaphragm position must be finite");
    double lam = 0.0, side[2][5];
    const int rc = riemann_sides(s->dim, s->gamma, s->gamma2, s->species, s->lambda_set, s->cfl, L, R, &lam,
                                 side);
    if (rc != LB_OK) return rc;
    s->lambda = lam;
    const double dx = (s->grid.x_hi - s->grid.x_lo) / (double)s->grid.nx;
    hipError_t e;
    if (s->precision == LB_FP64)
        e = launch_init_riemann<double>((double*)buf_ptr(s, 0), s->g, s->nf, s->grid.x_lo, dx, x_d,
                                        side[0], side[1], s->stream);
    else
        e = launch_init_riemann<float>((float*)buf_ptr(s, 0), s->g, s->nf, s->grid.x_lo, dx, x_d,
                                       side[0], side[1], s->stream);
    if (e != hipSuccess) return hip_fail(e, "init kernel");
    return start_state(s);
}

int lb_init_moments(lb_solver* s, const double* Y, double lambda)
{
    if (!s || !s->bound) return fail(LB_EINVAL, "solver not bound");
    if (!(lambda > 0.0) || !isfinite(lambda)) return fail(LB_EINVAL, "lambda must be > 0");
    int rc = check_moments(Y, s->nf, s->nn);
    if (rc != LB_OK) return rc;
    if (s->species && (rc = check_species(Y, s->nf, s->nn)) != LB_OK) return rc;
    rc = upload_moments(buf_ptr(s, 0), Y, s->nf, s->dim + 1, s->nn, lambda, s->precision == LB_FP64, s->stream);
    if (rc != LB_OK) return rc;
    s->lambda = lambda;
    return start_state(s);
}

// Queue n steps: step kernel + finalize kernel each.  With ev != NULL,
// ev[2i] / ev[2i+1] are recorded right before / after step i's step kernel.
static int queue_steps(lb_solver* s, int64_t n, hipEvent_t* ev = nullptr)
{
    for (int64_t i = 0; i < n; ++i) {
        const int in = s->cur, out = s->cur ^ 1;
        const long long step = (long long)(s->steps_done + 1);
        hipError_t e;
        if (ev && (e = hipEventRecord(ev[2 * i], s->stream)) != hipSuccess) return hip_fail(e, "event");
        if (s->dim == 1) {
            if (s->precision == LB_FP64)
                e = launch_step1d<double>((const double*)buf_ptr(s, in), (double*)buf_ptr(s, out), s->g,
                                          s->k, ctl_ptr(s), partials_ptr(s), step, s->stream);
            else
                e = launch_step1d<float>((const float*)buf_ptr(s, in), (float*)buf_ptr(s, out), s->g,
                                         s->k, ctl_ptr(s), partials_ptr(s), step, s->stream);
        } else if (s->hex) {
            if (s->precision == LB_FP64)
                e = launch_hex<double>((const double*)buf_ptr(s, in), (double*)buf_ptr(s, out), s->g, s->k,
                                       ctl_ptr(s), partials_ptr(s), step, s->stream);
            else
                e = launch_hex<float>((const float*)buf_ptr(s, in), (float*)buf_ptr(s, out), s->g, s->k,
                                      ctl_ptr(s), partials_ptr(s), step, s->stream);
        } else {
            if (s->precision == LB_FP64)
                e = launch_march2d<double>((const double*)buf_ptr(s, in), (double*)buf_ptr(s, out), s->g,
                                           s->march, s->k, ctl_ptr(s), partials_ptr(s), flags_ptr(s), step,
                                           s->stream, true);
            else
                e = launch_march2d<float>((const float*)buf_ptr(s, in), (float*)buf_ptr(s, out), s->g,
                                          s->march, s->k, ctl_ptr(s), partials_ptr(s), flags_ptr(s), step,
                                          s->stream, true);
        }
        if (e != hipSuccess) return hip_fail(e, "step launch");
        if (ev && (e = hipEventRecord(ev[2 * i + 1], s->stream)) != hipSuccess) return hip_fail(e, "event");
        e = launch_finalize(partials_ptr(s), s->nblocks, ctl_ptr(s), step, s->stream,
                            s->dim == 2 && s->species);
        if (e != hipSuccess) return hip_fail(e, "finalize launch");
        s->cur = out;
        s->steps_done += 1;
    }
    return LB_OK;
}

int lb_step(lb_solver* s, int64_t n)
{
    if (!s || !s->initialized) return fail(LB_EINVAL, "solver not initialised");
    if (n < 0) return fail(LB_EINVAL, "n must be >= 0");
    if (s->pending_err) return fail(s->pending_err, "an earlier step failed; re-initialise");
    return queue_steps(s, n);
}

// Wait, then roll the host view back to the last good step if one failed.
int lb_sync(lb_solver* s)
{
    if (!s || !s->bound) return fail(LB_EINVAL, "solver not bound");
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "sync");
    if (s->pending_err) return fail(s->pending_err, "an earlier step failed; re-initialise");
    if (!s->initialized) return LB_OK;
    StepCtl c;
    if ((e = hipMemcpy(&c, ctl_ptr(s), sizeof c, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "read control block");
    if (c.err_code) {
        // step err_step (1-based since init) failed; its input, the state
        // after err_step - 1 steps, sits in buffer (err_step - 1) & 1.
        const int64_t good = (int64_t)c.err_step - 1;
        s->steps_done = good;
        s->cur = (int)(good & 1);
        s->pending_err = (c.err_code & kErrState) ? LB_ESTATE : LB_EREACH;
        return fail(s->pending_err, "step %lld failed: %s", (long long)c.err_step,
                    (c.err_code & kErrState) ? "rho <= 0 or non-finite moment"
                                             : "a packet moves further than the halo");
    }
    return LB_OK;
}

int lb_step_timed(lb_solver* s, int64_t n, float* ms)
{
    if (!s || !ms) return fail(LB_EINVAL, "null argument");
    if (!s->initialized) return fail(LB_EINVAL, "solver not initialised");
    if (n < 0) return fail(LB_EINVAL, "n must be >= 0");
    if (s->pending_err) return fail(s->pending_err, "an earlier step failed; re-initialise");
    hipError_t e;
    if ((e = hipEventRecord(s->ev0, s->stream)) != hipSuccess) return hip_fail(e, "event");
    int rc = queue_steps(s, n);
    if (rc != LB_OK) return rc;
    if ((e = hipEventRecord(s->ev1, s->stream)) != hipSuccess) return hip_fail(e, "event");
    if ((e = hipEventSynchronize(s->ev1)) != hipSuccess) return hip_fail(e, "event sync");
    float t = 0.f;
    if ((e = hipEventElapsedTime(&t, s->ev0, s->ev1)) != hipSuccess) return hip_fail(e, "elapsed");
    rc = lb_sync(s);
    if (rc != LB_OK) return rc;
    *ms = t;
    return LB_OK;
}

int lb_step_profiled(lb_solver* s, int64_t n, float* kernel_ms, float* total_ms)
{
    if (!s || !kernel_ms || !total_ms) return fail(LB_EINVAL, "null argument");
    if (!s->initialized) return fail(LB_EINVAL, "solver not initialised");
    if (n < 0 || n > 100000) return fail(LB_EINVAL, "n must be in [0, 100000]");
    if (s->pending_err) return fail(s->pending_err, "an earlier step failed; re-initialise");
    std::vector<hipEvent_t> ev;
    try { ev.resize((size_t)(2 * n)); } catch (...) { return fail(LB_ENOMEM, "host alloc"); }
    hipError_t e;
    int rc = LB_OK;
    size_t made = 0;
    for (; made < ev.size(); ++made)
        if ((e = hipEventCreate(&ev[made])) != hipSuccess) { rc = hip_fail(e, "hipEventCreate"); break; }
    if (rc == LB_OK && (e = hipEventRecord(s->ev0, s->stream)) != hipSuccess) rc = hip_fail(e, "event");
    if (rc == LB_OK) rc = queue_steps(s, n, ev.data());
    if (rc == LB_OK && (e = hipEventRecord(s->ev1, s->stream)) != hipSuccess) rc = hip_fail(e, "event");
    if (rc == LB_OK && (e = hipEventSynchronize(s->ev1)) != hipSuccess) rc = hip_fail(e, "event sync");
    float kt = 0.f, tt = 0.f;
    for (int64_t i = 0; rc == LB_OK && i < n; ++i) {
        float t = 0.f;
        if ((e = hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1])) != hipSuccess) rc = hip_fail(e, "elapsed");
        kt += t;
    }
    if (rc == LB_OK && (e = hipEventElapsedTime(&tt, s->ev0, s->ev1)) != hipSuccess) rc = hip_fail(e, "elapsed");
    for (size_t i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
    if (rc != LB_OK) return rc;
    rc = lb_sync(s);
    if (rc != LB_OK) return rc;
    *kernel_ms = kt;
    *total_ms = tt;
    return LB_OK;
}

int lb_moments(lb_solver* s, double* out, int32_t on_device)
{
    if (!s || !out) return fail(LB_EINVAL, "null argument");
    if (!s->initialized) return fail(LB_EINVAL, "solver not initialised");
    int rc = lb_sync(s);
    if (rc != LB_OK && rc != LB_EREACH && rc != LB_ESTATE) return rc;
    // After a failed step the state is the last good one; exporting it is allowed.
    double sc[5];
    field_scales(s->nf, s->dim + 1, s->lambda, sc);
    double* dst = on_device ? out : export_ptr(s);
    hipError_t e = s->precision == LB_FP64
        ? launch_export<double>((const double*)buf_ptr(s, s->cur), dst, s->nn, s->nf, sc, s->stream)
        : launch_export<float>((const float*)buf_ptr(s, s->cur), dst, s->nn, s->nf, sc, s->stream);
    if (e != hipSuccess) return hip_fail(e, "export kernel");
    if (!on_device) {
        e = hipMemcpyAsync(out, dst, (size_t)s->nf * s->nn * 8, hipMemcpyDeviceToHost, s->stream);
        if (e != hipSuccess) return hip_fail(e, "copy out");
    }
    if ((e = hipStreamSynchronize(s->stream)) != hipSuccess) return hip_fail(e, "sync");
    if (rc != LB_OK) return fail(rc, "%s", "state is the last good step; an earlier step failed");
    return LB_OK;
}

// Interior sums of the device fields (lattice units) of the latest state:
// the step's own totals, or (no step since init) a host sum of the state.
static int field_totals(lb_solver* s, double t[5])
{
    if (!s->initialized) return fail(LB_EINVAL, "solver not initialised");
    int rc = lb_sync(s);
    if (rc != LB_OK) return rc;
    StepCtl c;
    hipError_t e = hipMemcpy(&c, ctl_ptr(s), sizeof c, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read control block");
    for (int f = 0; f < 5; ++f) t[f] = 0.0;
    if (c.totals_step == (long long)s->steps_done && s->steps_done > 0) {
        for (int f = 0; f < 4; ++f) t[f] = c.totals[f];
        if (s->nf == 5) t[4] = c.totals_sp;
    } else {
        // no step since init: sum the exported state on the host (index order)
        std::vector<double> y;
        try { y.resize((size_t)s->nf * s->nn); } catch (...) { return fail(LB_ENOMEM, "host alloc"); }
        double sc1[5] = {1, 1, 1, 1, 1};
        e = s->precision == LB_FP64
            ? launch_export<double>((const double*)buf_ptr(s, s->cur), export_ptr(s), s->nn, s->nf, sc1, s->stream)
            : launch_export<float>((const float*)buf_ptr(s, s->cur), export_ptr(s), s->nn, s->nf, sc1, s->stream);
        if (e != hipSuccess) return hip_fail(e, "export kernel");
        e = hipMemcpyAsync(y.data(), export_ptr(s), y.size() * 8, hipMemcpyDeviceToHost, s->stream);
        if (e != hipSuccess) return hip_fail(e, "copy out");
        if ((e = hipStreamSynchronize(s->stream)) != hipSuccess) return hip_fail(e, "sync");
        for (int f = 0; f < s->nf; ++f) {
            double a = 0.0;
            for (int64_t q = 0; q < s->nn; ++q) a += y[(size_t)f * s->nn + q];
            t[f] = a;
        }
    }
    return LB_OK;
}

int lb_totals(lb_solver* s, double out[4])
{
    if (!s || !out) return fail(LB_EINVAL, "null argument");
    double t[5];
    const int rc = field_totals(s, t);
    if (rc != LB_OK) return rc;
    double sc[5];
    field_scales(s->nf, s->dim + 1, s->lambda, sc);
    // field order on the device: rho, rho u, (rho v), rho E (, rho chi) -> out[0..3]
    double o[4] = {0, 0, 0, 0};
    o[0] = t[0] / sc[0];
    o[1] = t[1] / sc[1];
    if (s->dim == 2) {
        o[2] = t[2] / sc[2];
        o[3] = t[3] / sc[3];
    } else {
        o[3] = t[2] / sc[2];
    }
    for (int f = 0; f < 4; ++f) out[f] = o[f];
    return LB_OK;
}

int lb_species_total(lb_solver* s, double* out)
{
    if (!s || !out) return fail(LB_EINVAL, "null argument");
    if (!s->species) return fail(LB_EINVAL, "the solver has one gas");
    double t[5];
    const int rc = field_totals(s, t);
    if (rc != LB_OK) return rc;
    *out = t[s->nf - 1];  // rho chi needs no unit conversion
    return LB_OK;
}

double lb_lambda(const lb_solver* s) { return s ? s->lambda : 0.0; }

double lb_dt(const lb_solver* s)
{
    return s ? s->lambda * (s->grid.x_hi - s->grid.x_lo) / (double)s->grid.nx : 0.0;
}

int64_t lb_steps_done(const lb_solver* s) { return s ? s->steps_done : 0; }

int32_t lb_max_reach(lb_solver* s)
{
    if (!s || !s->bound) return -1;
    if (hipStreamSynchronize(s->stream) != hipSuccess) return -1;
    StepCtl c;
    if (hipMemcpy(&c, ctl_ptr(s), sizeof c, hipMemcpyDeviceToHost) != hipSuccess) return -1;
    return c.max_reach;
}

int lb_debug_lanes(lb_solver* s, int32_t* fx, int32_t* fy, int32_t* c1)
{
    if (!s || !fx || !fy || !c1) return fail(LB_EINVAL, "null argument");
    if (!s->initialized) return fail(LB_EINVAL, "solver not initialised");
    int rc = lb_sync(s);
    if (rc != LB_OK && rc != LB_EREACH && rc != LB_ESTATE) return rc;
    int32_t* d = (int32_t*)export_ptr(s);  // 3 nn int32 fit in the nf nn FP64 staging area
    hipError_t e = s->precision == LB_FP64
        ? launch_lanes<double>((const double*)buf_ptr(s, s->cur), s->g, s->dim, s->k, d, d + s->nn,
                               d + 2 * s->nn, s->stream)
        : launch_lanes<float>((const float*)buf_ptr(s, s->cur), s->g, s->dim, s->k, d, d + s->nn,
                              d + 2 * s->nn, s->stream);
    if (e != hipSuccess) return hip_fail(e, "lanes kernel");
    int32_t* outs[3] = {fx, fy, c1};
    for (int i = 0; i < 3; ++i) {
        e = hipMemcpyAsync(outs[i], d + (size_t)i * s->nn, (size_t)s->nn * 4, hipMemcpyDeviceToHost,
                           s->stream);
        if (e != hipSuccess) return hip_fail(e, "copy out");
    }
    if ((e = hipStreamSynchronize(s->stream)) != hipSuccess) return hip_fail(e, "sync");
    return LB_OK;
}

// ---- allocation-free stepping: lb_step_static ----
//
// The step kernels' scratch (control block, per-tile partial rows, tile flags)
// lives in the file-scope device array below instead of a bound buffer.  In
// host code `scratch` only stands in for the symbol: its device address, which
// differs per GPU, comes from hipGetSymbolAddress, taken once per device with
// that device current and kept in g_static.

}  // extern "C"

namespace {

constexpr size_t kStaticScratchBytes = (size_t)2 << 20;  // per device
constexpr size_t kStaticCtlBytes = 256;                  // the StepCtl at the front
static_assert(sizeof(StepCtl) <= kStaticCtlBytes, "control block must fit its slot");
constexpr int kStaticMaxDevices = 64;

struct StaticDevice {
    char* ptr = nullptr;  // device address of `scratch` on this device
    int cus = 0;          // compute units
    int per_cu[2] = {0, 0};       // resident blocks per CU of the square lattice's short pass, FP64 and FP32
    int per_cu_lean[2] = {0, 0};  // and of its lean pass
    bool ready = false;
};

std::mutex g_static_mu;
StaticDevice g_static[kStaticMaxDevices];

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

// Set-up of the current device (its first lb_step_static call): the address
// of its copy of `scratch`, its CU count and the march's occupancy.
int static_device(StaticDevice** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kStaticMaxDevices) return fail(LB_EINVAL, "device %d beyond %d", dev, kStaticMaxDevices);
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticDevice& d = g_static[dev];
    if (!d.ready) {
        void* p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess)
            return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if ((e = hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
            return hip_fail(e, "hipDeviceGetAttribute");
        d.per_cu[0] = march2d_blocks_per_cu<double>(false);
        d.per_cu[1] = march2d_blocks_per_cu<float>(false);
        d.per_cu_lean[0] = march2d_blocks_per_cu<double>(true);
        d.per_cu_lean[1] = march2d_blocks_per_cu<float>(true);
        d.ptr = (char*)p;
        d.ready = true;
    }
    *out = &d;
    return LB_OK;
}

bool is_device_ptr(const void* p)
{
    hipPointerAttribute_t attr;
    const hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice;
}

}  // namespace

extern "C" {

int lb_step_static(lb_solver* s, const void* Y_in, void* Y_out, void* hip_stream, int32_t* status_dev)
{
    if (!s || !Y_in || !Y_out) return fail(LB_EINVAL, "null argument");
    const size_t set = (size_t)s->nf * (size_t)s->nn * s->elem;
    const uintptr_t a = (uintptr_t)Y_in, b = (uintptr_t)Y_out;
    if (a % 256 != 0 || b % 256 != 0) return fail(LB_EINVAL, "moment buffers must be 256-byte aligned");
    if (a < b + set && b < a + set) return fail(LB_EINVAL, "input and output moment buffers overlap");
    if (!is_device_ptr(Y_in) || !is_device_ptr(Y_out) || (status_dev && !is_device_ptr(status_dev)))
        return fail(LB_EINVAL, "buffers must be device memory");
    StaticDevice* d = nullptr;
    int rc = static_device(&d);
    if (rc != LB_OK) return rc;
    // scratch layout: control block, partial rows (one per block / tile), tile flags (two words per tile)
    MarchGeom m{};
    int64_t rows = 0;
    const bool march = s->dim == 2 && !s->hex;  // the square lattice's passes (tile flags)
    if (s->dim == 1) {
        rows = step_blocks_1d(s->g);
    } else if (s->hex) {
        rows = hex_blocks(s->g);
    } else {
        const int pi = s->precision == LB_FP64 ? 0 : 1;
        m = march2d_geometry(s->g, d->cus, d->per_cu[pi], d->per_cu_lean[pi]);
        rows = m.blocks();
    }
    const size_t part_bytes = align256((size_t)rows * kPartialStride * 8);
    const size_t need = kStaticCtlBytes + part_bytes + (march ? align256((size_t)rows * 2 * 4) : 0);
    if (need > kStaticScratchBytes)
        return fail(LB_EINVAL, "grid %lld x %lld needs %zu bytes of step scratch, more than the %zu of lb_step_static",
                    (long long)s->g.nx, (long long)s->g.ny, need, kStaticScratchBytes);
    StepCtl* ctl = (StepCtl*)d->ptr;
    double* partials = (double*)(d->ptr + kStaticCtlBytes);
    int* flags = (int*)(d->ptr + kStaticCtlBytes + part_bytes);
    const hipStream_t st = (hipStream_t)hip_stream;
    // the last call's control block is stale: a fill kernel resets it (no
    // memset, so the call can be captured into a graph)
    hipError_t e = launch_reset_ctl(ctl, st);
    if (e == hipSuccess && march) e = launch_fill_i32(flags, 2 * rows, 0, st);  // the last call's flags
    if (e != hipSuccess) return hip_fail(e, "reset");
    if (s->dim == 1) {
        e = s->precision == LB_FP64
            ? launch_step1d<double>((const double*)Y_in, (double*)Y_out, s->g, s->k, ctl, partials, 1, st)
            : launch_step1d<float>((const float*)Y_in, (float*)Y_out, s->g, s->k, ctl, partials, 1, st);
    } else if (s->hex) {
        e = s->precision == LB_FP64
            ? launch_hex<double>((const double*)Y_in, (double*)Y_out, s->g, s->k, ctl, partials, 1, st)
            : launch_hex<float>((const float*)Y_in, (float*)Y_out, s->g, s->k, ctl, partials, 1, st);
    } else {
        e = s->precision == LB_FP64
            ? launch_march2d<double>((const double*)Y_in, (double*)Y_out, s->g, m, s->k, ctl, partials, flags, 1, st,
                                     false)
            : launch_march2d<float>((const float*)Y_in, (float*)Y_out, s->g, m, s->k, ctl, partials, flags, 1, st,
                                    false);
    }
    if (e != hipSuccess) return hip_fail(e, "step launch");
    if ((e = launch_finalize(partials, rows, ctl, 1, st, s->dim == 2 && s->species)) != hipSuccess)
        return hip_fail(e, "finalize launch");
    if (status_dev && (e = launch_status(ctl, status_dev, st)) != hipSuccess) return hip_fail(e, "status launch");
    return LB_OK;
}

void lb_destroy(lb_solver* s)
{
    if (!s) return;
    if (s->bound) (void)hipStreamSynchronize(s->stream);
    if (s->events) {
        (void)hipEventDestroy(s->ev0);
        (void)hipEventDestroy(s->ev1);
    }
    delete s;
}

}  // extern "C"
