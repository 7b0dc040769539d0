/*
 * lbsd -- C ABI of the semi-discrete compressible lattice Boltzmann step
 * (tau = 1) of Komeili, Mirzaei and Shabouei, "Performance of 1-D and 2-D
 * Lattice Boltzmann (LB) in Solution of the Shock Tube Problem"
 * (arXiv 1602.02675), on AMD Instinct MI355X (gfx950).
 *
 * The calls follow the paper's own statement of the problem (Sec. V.A): set
 * the initial flow parameters (density, velocity, energy), advance the
 * migration step, read the moments back.
 *
 * Conventions
 *  - Every call returns an int status (LB_OK = 0, negative on error) unless
 *    stated otherwise; out-parameters are written only on LB_OK (one
 *    exception: lb_moments, see there); nothing throws across the ABI.  lb_last_error() gives a message for the calling
 *    thread's last failed call.
 *  - Device memory is owned by the caller: lb_state_bytes() says how much,
 *    lb_bind() hands over a device pointer (e.g. a PyTorch tensor's
 *    data_ptr()) and a HIP stream.  The caller keeps that memory alive until
 *    lb_destroy().  The library owns the handle.
 *  - Device work is stream-ordered on the bound stream.  lb_step() returns
 *    as soon as the launches are queued; errors detected on the device
 *    (LB_EREACH, LB_ESTATE) are reported by the next call that synchronises
 *    (lb_sync, lb_moments, lb_totals, lb_step_timed).
 *  - One handle is not thread-safe; different handles on different streams
 *    may run concurrently.
 *  - Units: the caller speaks physical units.  Inside, the lattice spacing
 *    and time step are 1 and lambda = dt/dx scales velocity (x lambda) and
 *    energy per unit mass (x lambda^2).
 */
#ifndef LBSD_H
#define LBSD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define LB_OK 0
#define LB_EINVAL (-1)  /* bad argument: size, gamma outside (1, 1 + 2/D], delta0 outside [0, 1), n < 0 ... */
#define LB_ENOMEM (-2)  /* bound buffer too small / host allocation failed */
#define LB_EDEVICE (-3) /* a HIP call failed */
#define LB_ESTATE (-4)  /* rho <= 0, p < 0 or a non-finite value in a state */
#define LB_EREACH (-5)  /* a packet would move further than the halo (LB_HALO nodes) in one step */

/* ---- enumerations ---- */
#define LB_BC_TRANSMISSIVE 0 /* ghost nodes copy the edge node every step; packets leaving are dropped (Sec. V.B) */
#define LB_BC_PERIODIC 1     /* the lateral direction of the 2-D lattice (Sec. V.B); also allowed along x */
#define LB_BC_REFLECTING 2   /* a wall on the outer face of each edge node reflects crossing packets
                              * specularly: normal momentum negated, mass and energy kept (the shock
                              * reflection the conclusions name as an extension); needs n >= LB_HALO
                              * along that axis */

#define LB_LATTICE_D1_TRIPLE 1       /* 1-D triple-level set (Sec. IV.A): c' in {0, +-c'_1, +-c'_2}, b0=1, b1=b2=2 */
#define LB_LATTICE_D2_SQUARE_DUAL 2  /* square dual-level set (Sec. IV.B): +-c'_1, +-c'_2 along x and y, d0=0, b1=b2=4 */
#define LB_LATTICE_D2_SQUARE_TRIPLE 3 /* square set with a rest level: the dual-level set plus one rest group,
                                       * b0=1, d0 = d0_frac rho, d0_frac in (0, 1) (eq. 24-26 with b_0 d_0;
                                       * the paper's square lattice takes d0 = 0) */
#define LB_LATTICE_D2_HEX_DUAL 4     /* hexagonal lattice (Fig. 1, Sec. III.B with b_v = 6): six directions 60 degrees
                                      * apart at c'_1 and c'_2, d0 = 0, b1 = b2 = 6.  Nodes at i e_1 + j e_2 with
                                      * e_1 = (1, 0), e_2 = (1/2, sqrt(3)/2) (x spacing dx), stored [f][j][i];
                                      * momenta are Cartesian; bc_x / bc_y apply to the axial indices i / j
                                      * (transmissive or periodic; no walls, one gas).  A velocity's end point
                                      * lies in a lattice triangle whose three nodes take its barycentric weights */
#define LB_LATTICE_D2_HEX_TRIPLE 5   /* the hexagonal set plus one rest group, b0 = 1, d0 = d0_frac rho, d0_frac in (0, 1) */

#define LB_FP64 0 /* FP64 storage and arithmetic */
#define LB_FP32 1 /* FP32 storage and arithmetic, FP64 conservation totals */

#define LB_HALO 5 /* largest per-axis displacement a packet may have in one step */

typedef struct lb_solver lb_solver; /* opaque */

/* Grid: dim 1 -> ny must be 1.  Nodes are cell centres x_i = x_lo + (i + 1/2) dx,
 * dx = (x_hi - x_lo) / nx; the square lattice has dy = dx (the hexagonal one
 * rows sqrt(3)/2 dx apart, row j shifted by j dx / 2; lb_init_riemann splits it
 * by the axial index i, i.e. along lines parallel to e_2).  Limits: nx, ny
 * <= 2^40, nx ny <= 2^36, and nx <= 2^28 on the 2-D lattices (LB_EINVAL). */
typedef struct {
    int32_t dim;
    int64_t nx, ny;
    double x_lo, x_hi;
    int32_t bc_x, bc_y;
} lb_grid;

/* Velocity set: lattice (must match dim) and d0_frac = d_0 / rho, the rest
 * weight of the triple-level sets (the paper picks 0.4 .. 0.55 in 1-D; 0.5 is
 * the usual choice); must be 0 for the square dual-level set. */
typedef struct {
    int32_t lattice;
    double d0_frac;
} lb_velset;

/* Primitive state in physical units; v is ignored in 1-D. */
typedef struct {
    double rho, u, v, p;
} lb_prim;

/* Create a solver for one grid (Sec. III-IV).  gamma must lie in (1, 1 + 2/D]
 * so that the non-translational energy phi of eq. 15 is non-negative.
 * precision: LB_FP64 or LB_FP32.  *out receives the handle. */
int lb_create(const lb_grid* grid, double gamma, const lb_velset* velset, int32_t precision,
              lb_solver** out);

/* Two gases (the different gases on the two sides of the tube that the
 * conclusions name as an extension), on every lattice: gas 1 with gamma_1 and gas 2 with gamma_2, both ideal with
 * one gas constant, each in (1, 1 + 2/D].  The state gains a species moment
 * rho chi (chi = mass fraction of gas 1) after rho E (nf = dim + 3); every
 * packet carries its source's chi as it carries its mass, and a node's gas is
 * the mixture by mass fraction:
 * gamma - 1 = 1 / (chi / (gamma_1 - 1) + (1 - chi) / (gamma_2 - 1)), which
 * sets phi (eq. 15) and the level speeds (eq. 26).  lb_init_riemann puts gas 1
 * on the left and gas 2 on the right (rho E and the CFL speed of each side
 * from its own gamma); lb_init_moments and lb_moments take and give all
 * fields.  With the rest level of LB_LATTICE_D2_SQUARE_TRIPLE, d_0 = d0_frac
 * rho carries chi too. */
int lb_create_two_gas(const lb_grid* grid, double gamma_1, double gamma_2, const lb_velset* velset,
                      int32_t precision, lb_solver** out);

/* Bytes of device memory the solver needs (two ping-pong SoA moment sets,
 * export staging, control block, per-block partials). */
size_t lb_state_bytes(const lb_solver* s);

/* Hand over device memory (>= lb_state_bytes, 256-byte aligned) and the HIP
 * stream (hipStream_t, NULL = default stream) all later work is queued on. */
int lb_bind(lb_solver* s, void* dev_ptr, size_t bytes, void* hip_stream);

/* lambda = dt/dx used by the next lb_init_* call: the kernel works in lattice
 * units (dx = dt = 1, Sec. III), so velocities scale by lambda and energies per
 * unit mass by lambda^2.  The paper states no time step; lb_set_lambda fixes
 * it (> 0); lb_set_cfl (> 0, default 1) makes lb_init_riemann take
 * lambda = cfl / max(|u| + sqrt(gamma p / rho)) over the two states, the
 * reading that a CFL number of 1 on the initial states sets dt (the fastest
 * initial signal then moves at most one node per step). */
int lb_set_lambda(lb_solver* s, double lambda);
int lb_set_cfl(lb_solver* s, double cfl);

/* Riemann problem (Sec. V.C): node i gets `left` when x_i < x_diaphragm, else
 * `right`; rho E = p/(gamma - 1) + rho |u|^2 / 2 (eq. 27).  Resets the step
 * count and any pending error.  LB_ESTATE for rho <= 0, p < 0, non-finite. */
int lb_init_riemann(lb_solver* s, double x_diaphragm, const lb_prim* left, const lb_prim* right);

/* General initial state: host_Y is FP64 SoA [nf][ny][nx] of the conserved
 * moments rho, rho u, (rho v), rho E (, rho chi with two gases) in physical
 * units (nf = dim + 2, or dim + 3 with two gases), and lambda > 0 the time-step
 * ratio to use.  Copied synchronously.  LB_ESTATE for rho <= 0, a
 * non-finite value, or (two gases) rho chi outside [0, rho]. */
int lb_init_moments(lb_solver* s, const double* host_Y, double lambda);

/* Queue n >= 0 steps (eq. 10 / eq. 30 with tau = 1, Sec. V.A).  Each step
 * queues its step launches on the bound stream -- one kernel in 1-D and on the
 * hexagonal lattice; on the square lattice a first pass over the tiles, and
 * two further passes that return at once unless the earlier pass left tiles
 * to them -- and then a small kernel that reduces the per-tile partial
 * results into the interior conservation totals and the largest reach.  If a
 * step fails, it and every later queued step leave the state at the last good
 * step; the error is reported at the next synchronising call. */
int lb_step(lb_solver* s, int64_t n);

/* As lb_step, bracketed by HIP events on the bound stream; waits and writes
 * the elapsed milliseconds of the n steps to *ms. */
int lb_step_timed(lb_solver* s, int64_t n, float* ms);

/* As lb_step_timed, with HIP events also around each step kernel (not its
 * small totals-reduction kernel): *kernel_ms gets the summed duration of the
 * n step kernels, *total_ms the elapsed time of the whole sequence.  n <= 100000. */
int lb_step_profiled(lb_solver* s, int64_t n, float* kernel_ms, float* total_ms);

/* Wait for queued work; returns LB_EREACH / LB_ESTATE if a step failed. */
int lb_sync(lb_solver* s);

/* Current moments (eq. 6-7: rho, rho v and rho E, the sums of eq. 22 over
 * the packets that landed on each node) as FP64 SoA [nf][ny][nx] in physical
 * units, into `out` (host memory, or device memory when out_on_device != 0);
 * the primitives of Sec. V.D follow from them (u = rho u / rho, e = E - u^2/2,
 * p by eq. 27).  Synchronises.
 * After a failed step (LB_EREACH, LB_ESTATE) it still writes `out`: the
 * state of the last good step, which the failed step left intact, and
 * returns that step's error. */
int lb_moments(lb_solver* s, double* out, int32_t out_on_device);

/* Interior sums of rho, rho u, rho v (0 in 1-D), rho E of the current state
 * in physical units per node (multiply by dx for integrals).  Each node's
 * packets carry its mass, momentum and energy exactly (eq. 22), so these are
 * conserved to rounding while nothing crosses a boundary (periodic, walls),
 * and change only by the flux through transmissive ends (Sec. V.B).  The step
 * kernels form them in FP64 with a fixed reduction order.  Synchronises. */
int lb_totals(lb_solver* s, double out[4]);

/* Two gases: interior sum of rho chi (the mass of gas 1 per dx) of the
 * current state, as lb_totals forms it.  LB_EINVAL for a one-gas solver. */
int lb_species_total(lb_solver* s, double* out);

double lb_lambda(const lb_solver* s);         /* lambda of the current state (0 before init) */
double lb_dt(const lb_solver* s);             /* physical time step lambda * dx */
int64_t lb_steps_done(const lb_solver* s);    /* good steps since the last init */
int32_t lb_max_reach(lb_solver* s);           /* largest reach of the latest step (synchronises) */

/* Per-node floor(v_x), floor(v_y) (0 in 1-D) and c'_1 (eq. 26) of the current
 * state, computed by the same device function the step uses; host int32
 * arrays of nx*ny entries.  Synchronises. */
int lb_debug_lanes(lb_solver* s, int32_t* floor_x, int32_t* floor_y, int32_t* c1);

void lb_destroy(lb_solver* s);
const char* lb_last_error(void);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one step
 * of solver s's problem (grid, gamma, velocity set, precision; s needs no
 * lb_bind) from the moment fields Y_in to Y_out, without the bound buffer.
 * Y_in and Y_out are device SoA arrays [nf][ny][nx] in the storage type
 * (double for LB_FP64, float for LB_FP32) in lattice units: rho,
 * rho u lambda, (rho v lambda), rho E lambda^2 (, rho chi); each 256-byte
 * aligned, not overlapping.  The caller owns both; Y_in is only read.  The
 * step's scratch (control block, per-tile partial sums, tile flags) is a
 * static device array of 2 MiB per GPU, which the library holds until the
 * process ends; grids that need more are rejected with LB_EINVAL (1-D tubes
 * above about 33 M nodes; a 2-D grid is cut into about three tiles per
 * resident block whatever its size, and only grids wider than about 7 M
 * columns need more).
 * The call queues kernels on hip_stream and returns; it calls no hipMalloc,
 * hipFree or allocating library routine.  If status_dev (a device int32, may
 * be NULL) is given, the stream writes LB_OK, LB_EREACH or LB_ESTATE to it
 * after the step; after a failure Y_out is unspecified and Y_in is the last
 * good state.  All calls on one GPU share its scratch array and reset it at
 * their start: calls whose work overlaps on one GPU (other streams, other
 * threads) race and must be serialised by the caller. */
int lb_step_static(lb_solver* s, const void* Y_in, void* Y_out, void* hip_stream, int32_t* status_dev);

/* ---- pools: many independent problems, one persistent launch per step ----
 *
 * The batching and serving forms.  A pool holds up to max_slots problems of one
 * lattice, gamma and precision (each with its own grid, lambda, boundary
 * conditions and step target) in an arena of arena_bytes inside the caller's
 * device memory.  One pool step is one kernel launch over a tile table in
 * device memory (square lattice: persistent blocks that claim tiles, plus a
 * pass that redoes the tiles whose packets reached past the short FIFO; 1-D:
 * one block per tile) and a per-slot reduction kernel; every live, unfinished
 * slot advances by one step (eq. 10 / 30 with tau = 1, as lb_step).
 * Admissions and releases rewrite the tables between launches, in stream
 * order: steps queued before them run with the old tables, steps queued
 * after with the new ones, and the host does not wait for the device (so a
 * serving loop can keep the next steps queued while it admits and releases).
 * On the square lattice the launch shape, and so a captured HIP graph, stays
 * valid while problems come and go (1-D re-captures when the number of tiles
 * changes).
 * A slot's results do not depend on what else is in the pool, the tile shape
 * or graph use: they are bit-identical to an lb_solver run of the same
 * problem.
 *
 * Slot status (lb_pool_poll): 0 running, 1 reached its step target, or
 * LB_EREACH / LB_ESTATE if one of its steps failed (it then stops at its last
 * good step; other slots go on).  Calls that synchronise: poll, status,
 * moments, totals, set_shape, autotune, admit_moments; snapshot_read waits
 * only for its snapshot. */
typedef struct lb_pool lb_pool; /* opaque */

/* max_slots in [1, 2^20]; arena_bytes: device memory for the slots' moment
 * sets (lb_pool_footprint per slot). */
int lb_pool_create(int32_t dim, double gamma, const lb_velset* velset, int32_t precision,
                   int32_t max_slots, size_t arena_bytes, lb_pool** out);
/* A pool of two-gas problems (as lb_create_two_gas: gas 1 gamma_1, gas 2
 * gamma_2, a species field rho chi after rho E in every slot; admission by
 * moments checks rho chi in [0, rho]).  lb_pool_totals reports the four
 * one-gas totals. */
int lb_pool_create_two_gas(int32_t dim, double gamma_1, double gamma_2, const lb_velset* velset,
                           int32_t precision, int32_t max_slots, size_t arena_bytes, lb_pool** out);
size_t lb_pool_bytes(const lb_pool* p);                   /* device bytes to bind (arena + tables) */
size_t lb_pool_footprint(const lb_pool* p, int64_t nx, int64_t ny); /* arena bytes one problem takes */
/* As lb_bind.  A non-default stream is required for lb_pool_use_graph. */
int lb_pool_bind(lb_pool* p, void* dev_ptr, size_t bytes, void* hip_stream);

/* Admit a Riemann problem (as lb_init_riemann; lambda <= 0 takes the CFL-1
 * rule) that stops after `steps` steps.  *slot receives its slot.  LB_ENOMEM
 * when no slot is free or its footprint does not fit the arena now. */
int lb_pool_admit_riemann(lb_pool* p, const lb_grid* grid, double lambda, double x_diaphragm,
                          const lb_prim* left, const lb_prim* right, int64_t steps, int32_t* slot);
/* Admit a general state (as lb_init_moments). */
int lb_pool_admit_moments(lb_pool* p, const lb_grid* grid, const double* host_Y, double lambda,
                          int64_t steps, int32_t* slot);
/* Free a slot and its arena space.  Does not wait: steps queued before the
 * release still advance the slot (into its own memory), and anything that
 * reuses that memory is queued after them. */
int lb_pool_release(lb_pool* p, int32_t slot);

/* Queue n >= 0 pool steps (async; graph launches when lb_pool_use_graph is on). */
int lb_pool_advance(lb_pool* p, int64_t n);
/* As lb_pool_advance, bracketed by HIP events on the bound stream; waits and
 * writes the elapsed milliseconds to *ms (a graph is captured before timing). */
int lb_pool_advance_timed(lb_pool* p, int64_t n, float* ms);

int lb_pool_poll(lb_pool* p, int32_t slot, int64_t* steps_done, int32_t* status);
/* lb_pool_poll for every slot at once: arrays of max_slots entries; a free
 * slot reports 0 steps and status LB_POOL_FREE. */
#define LB_POOL_FREE (-100)
int lb_pool_status(lb_pool* p, int64_t* steps_done, int32_t* status);
/* Progress snapshots for serving loops that keep steps queued: snapshot
 * queues, behind the work queued so far, a copy of every slot's progress
 * into host buffer `buf` (0 or 1) and returns at once; snapshot_read waits
 * for that copy only and gives, per slot (arrays of max_slots entries, totals
 * [max_slots][4] or NULL), steps done, the status of lb_pool_poll, and the
 * totals of lb_pool_totals (NaN before a slot's first step).  A slot that was
 * free when the snapshot was queued, or was released and admitted again
 * since, reports LB_POOL_FREE.  Queuing into a buffer whose previous snapshot
 * is still in flight waits for it. */
int lb_pool_snapshot(lb_pool* p, int32_t buf);
int lb_pool_snapshot_read(lb_pool* p, int32_t buf, int64_t* steps_done, int32_t* status, double* totals);
/* As lb_moments / lb_totals for one slot (lb_pool_totals: LB_EINVAL before its first step).
 * A slot whose step failed exports its last good state and returns LB_OK;
 * lb_pool_poll reports the failure. */
int lb_pool_moments(lb_pool* p, int32_t slot, double* out, int32_t out_on_device);
int lb_pool_totals(lb_pool* p, int32_t slot, double out[4]);
double lb_pool_lambda(const lb_pool* p, int32_t slot);
int32_t lb_pool_live(const lb_pool* p);                  /* admitted slots */

/* Tile shapes: 1-D, threads x nodes per thread in {256x1, 256x2, 256x4,
 * 256x8, 512x4}; square lattice, tiles of 246 columns whose strip height makes
 * about {2, 3, 4, 6, 8} tiles per resident block over the live problems (at
 * least 16 rows).  lb_pool_autotune times `trials` steps of every shape on the
 * admitted problems without changing their states, keeps the fastest and
 * writes its index and median milliseconds per step. */
int32_t lb_pool_shapes(const lb_pool* p);
int32_t lb_pool_shape(const lb_pool* p);
int lb_pool_set_shape(lb_pool* p, int32_t shape);
int lb_pool_autotune(lb_pool* p, int32_t trials, int32_t* best, float* ms_per_step);
/* Capture steps_per_graph pool steps as one HIP graph (0: plain launches). */
int lb_pool_use_graph(lb_pool* p, int32_t steps_per_graph);
void lb_pool_destroy(lb_pool* p);

#ifdef __cplusplus
}
#endif

#endif /* LBSD_H */
