// The tau = 1 step of the semi-discrete compressible LB method on the 1-D
// triple-level lattice as one fused gather kernel per step (Komeili, Mirzaei,
// Shabouei, arXiv 1602.02675, Sec. III-V), and the per-step reduction kernel
// shared with the square lattice (whose step kernel is in lb_march2d.hip).
//
// With tau = 1 the distribution after a step is the migrated equilibrium
// (eq. 10, eq. 30), and the equilibrium depends on the node moments only, so
// the whole state is the SoA moment field Y = (rho, rho v, rho E) (eq. 7) and a
// step maps Y to Y'.  Every node (source) emits packets m (1, v + c', zeta) to
// x + floor(v) + k + c' (eq. 11-13, 21, 23); Y' at a node is the sum of what
// lands there (Sec. V.A).
//
// GPU formulation (deterministic gather, no atomics on field data):
//   1. a block stages the sources of its destination tile plus a halo of H
//      nodes in LDS, reduced to (f, r, c'_1, d_v, K) per source
//      (lb_device.hpp);
//   2. every destination rebuilds each packet class (lane, corner) from the
//      source that class maps onto it.  In a tile where floor(v) and c'_1 are
//      the same for every staged source (the integer parts of the migration
//      vectors are piecewise constant), each class has exactly one source at
//      a compile-time offset, and the 10 packets are fully unrolled;
//      otherwise every candidate displacement in the tile's range is tested
//      against the source's own displacement;
//   3. the interior sums of the new moments are reduced per block with
//      wavefront shuffles into one row of per-block partials; a one-block
//      kernel then adds the rows in a fixed order (deterministic totals) and
//      records the reach (halo overflow) and state checks.
#include <climits>

#include "lb_kernels.hpp"

namespace lbsd {

namespace {

__device__ __forceinline__ int pack_lane(int fx, int fy, int c1)
{
    fx = fx < -127 ? -127 : (fx > 127 ? 127 : fx);
    fy = fy < -127 ? -127 : (fy > 127 ? 127 : fy);
    c1 = c1 > 255 ? 255 : c1;
    return (fx + 128) | ((fy + 128) << 8) | (c1 << 16);
}
__device__ __forceinline__ int lane_fx(int p) { return (p & 255) - 128; }
__device__ __forceinline__ int lane_fy(int p) { return ((p >> 8) & 255) - 128; }
__device__ __forceinline__ int lane_c1(int p) { return (p >> 16) & 255; }

// Integer summary of the staged sources of one block.
struct TileInfo {
    int fxmin, fxmax, fymin, fymax, cmin, cmax, reach, bad;
};

template <int NW>
__device__ __forceinline__ TileInfo block_tile_info(TileInfo t, int (*s_red)[8])
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    t.fxmin = wave_min(t.fxmin); t.fxmax = wave_max(t.fxmax);
    t.fymin = wave_min(t.fymin); t.fymax = wave_max(t.fymax);
    t.cmin = wave_min(t.cmin);   t.cmax = wave_max(t.cmax);
    t.reach = wave_max(t.reach); t.bad = wave_max(t.bad);
    if (lane == 0) {
        s_red[wid][0] = t.fxmin; s_red[wid][1] = t.fxmax;
        s_red[wid][2] = t.fymin; s_red[wid][3] = t.fymax;
        s_red[wid][4] = t.cmin;  s_red[wid][5] = t.cmax;
        s_red[wid][6] = t.reach; s_red[wid][7] = t.bad;
    }
    __syncthreads();
    TileInfo r = {s_red[0][0], s_red[0][1], s_red[0][2], s_red[0][3],
                  s_red[0][4], s_red[0][5], s_red[0][6], s_red[0][7]};
#pragma unroll
    for (int w = 1; w < NW; ++w) {
        r.fxmin = min(r.fxmin, s_red[w][0]); r.fxmax = max(r.fxmax, s_red[w][1]);
        r.fymin = min(r.fymin, s_red[w][2]); r.fymax = max(r.fymax, s_red[w][3]);
        r.cmin = min(r.cmin, s_red[w][4]);   r.cmax = max(r.cmax, s_red[w][5]);
        r.reach = max(r.reach, s_red[w][6]); r.bad = max(r.bad, s_red[w][7]);
    }
    return r;
}

// Epilogue: per-block field sums and checks -> one row of `partials`.  No
// atomics or device-scope fences here: the reduction over blocks is a separate
// single-block kernel (finalize_kernel), so the kernel boundary orders it.
template <int NW, int NF>
__device__ void finish_step(double (&acc)[NF], const TileInfo& ti, double* __restrict__ prow, int H)
{
    __shared__ double s_sum[NW][4];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = wave_sum(acc[f]);
    if (lane == 0) {
#pragma unroll
        for (int f = 0; f < NF; ++f) s_sum[wid][f] = acc[f];
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            double s = s_sum[0][f];
            for (int w = 1; w < NW; ++w) s += s_sum[w][f];
            prow[f] = s;
        }
        for (int f = NF; f < 4; ++f) prow[f] = 0.0;
        prow[4] = (double)ti.reach;
        prow[5] = (double)((ti.reach > H ? kErrReach : 0) | (ti.bad ? kErrState : 0));
    }
}

// First stage of the reduction of many partial rows (a 1-D step has one row
// per 1024 nodes, 16 K rows at 2^24 nodes, too many for one block to read
// quickly): block g folds rows [g kChunk, (g + 1) kChunk) in a fixed order
// (sums, largest reach, error bits) into row g kChunk, the first of its own
// chunk, so that blocks never touch each other's rows.
constexpr int kChunk = 256;
__global__ void __launch_bounds__(kChunk)
partials_chunk_kernel(double* __restrict__ partials, int64_t nb, const StepCtl* __restrict__ ctl, long long step)
{
    __shared__ double s_sum[kChunk / 64][5];
    __shared__ int s_ir[kChunk / 64][2];
    if (ctl->err_step < step) return;  // an earlier step failed: the rows are not this step's
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t b0 = (int64_t)blockIdx.x * kChunk, b = b0 + tid;
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    int reach = 0, err = 0;
    if (b < nb) {
        const double* p = partials + b * kPartialStride;
#pragma unroll
        for (int f = 0; f < 4; ++f) s[f] = p[f];
        s[4] = p[6];
        reach = (int)p[4];
        err = (int)p[5];
    }
#pragma unroll
    for (int f = 0; f < 5; ++f) s[f] = wave_sum(s[f]);
    reach = wave_max(reach);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) err |= __shfl_xor(err, o, 64);
    if (lane == 0) {
#pragma unroll
        for (int f = 0; f < 5; ++f) s_sum[wid][f] = s[f];
        s_ir[wid][0] = reach;
        s_ir[wid][1] = err;
    }
    __syncthreads();
    if (tid == 0) {
        double* q = partials + b0 * kPartialStride;
        for (int f = 0; f < 5; ++f) {
            double t = s_sum[0][f];
            for (int w = 1; w < kChunk / 64; ++w) t += s_sum[w][f];
            q[f < 4 ? f : 6] = t;
        }
        int r = s_ir[0][0], e = s_ir[0][1];
        for (int w = 1; w < kChunk / 64; ++w) { r = max(r, s_ir[w][0]); e |= s_ir[w][1]; }
        q[4] = (double)r;
        q[5] = (double)e;
    }
}

// Sum the per-block partials of one step in a fixed order (deterministic),
// record the totals, the largest reach and the first failed step.  Rows b
// stride for b < nb (stride > 1: the chunk heads of partials_chunk_kernel).
constexpr int kFinTPB = 256;
__global__ void __launch_bounds__(kFinTPB)
finalize_kernel(const double* __restrict__ partials, int64_t nb, int64_t stride, StepCtl* __restrict__ ctl,
                long long step, int sp2)
{
    __shared__ double s_sum[kFinTPB / 64][5];
    __shared__ int s_ir[kFinTPB / 64][2];
    if (threadIdx.x == 0) {  // the step kernels of this step are done with their counters
        for (int i = 0; i < 5; ++i) ctl->next[i] = 0;
        ctl->keep[1] = ctl->keep[0];
        ctl->keep[0] = 0;
        ctl->split_n[(step + 1) & 1] = 0;  // the next step lists its tiles afresh
        ctl->full_n = 0;
    }
    if (ctl->err_step < step) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    int reach = 0, err = 0;
    for (int64_t b = tid; b < nb; b += kFinTPB) {
        const double* p = partials + b * stride * kPartialStride;
#pragma unroll
        for (int f = 0; f < 4; ++f) s[f] += p[f];
        if (sp2) s[4] += p[6];  // rho chi (square lattice, two gases)
        reach = max(reach, (int)p[4]);
        err |= (int)p[5];
    }
#pragma unroll
    for (int f = 0; f < 5; ++f) s[f] = wave_sum(s[f]);
    reach = wave_max(reach);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) err |= __shfl_xor(err, o, 64);
    if (lane == 0) {
#pragma unroll
        for (int f = 0; f < 5; ++f) s_sum[wid][f] = s[f];
        s_ir[wid][0] = reach;
        s_ir[wid][1] = err;
    }
    __syncthreads();
    if (tid == 0) {
        for (int f = 0; f < 5; ++f) {
            double t = s_sum[0][f];
            for (int w = 1; w < kFinTPB / 64; ++w) t += s_sum[w][f];
            if (f < 4) ctl->totals[f] = t;
            else ctl->totals_sp = t;
        }
        int r = s_ir[0][0], e = s_ir[0][1];
        for (int w = 1; w < kFinTPB / 64; ++w) { r = max(r, s_ir[w][0]); e |= s_ir[w][1]; }
        ctl->max_reach = r;
        ctl->totals_step = step;
        if (e) {
            ctl->err_code = e;
            ctl->err_step = step;
        }
    }
}

// ------------------------------------------------------------------ 1-D ----

// The staged sources of a 1-D tile.  Of the level weights only d_2 is staged,
// with rho: d_0 = delta0 rho and d_1 = (rho - b_0 d_0) / b_1 - d_2 are formed
// again where a packet needs them, with the source's own expressions (the
// same values for FP64 storage), which keeps a tile's LDS small enough for a
// fourth block per CU.
template <typename T>
struct Tile1 {
    int* pk;
    T *r, *rho, *d2, *K;  // rho: 0 for a bad source (its packets are then empty)
    T* chi;  // two gases: mass fraction of gas 1 per source
    T delta0, b0, inv_b1;
};

// One packet of a 1-D source s at displacement k + c' from its floor node:
// mass alpha_k d, momentum m (v + c'), energy m (K + c' v + c'^2/2); with two
// gases (SP) also the species moment m chi.
template <typename T, bool SP>
__device__ __forceinline__ void add_packet1(const Tile1<T>& tl, int s, int f, int k, int lane_c,
                                            int lev, T& R, T& P, T& En, T& X)
{
#pragma clang fp contract(off)
    const T r = tl.r[s];
    const T a = k ? r : (T)1 - r;
    T d;
    if (lev == 2) {
        d = tl.d2[s];
    } else {
        const T rho = tl.rho[s];
        const T d0 = tl.delta0 * rho;
        d = lev == 0 ? d0 : (rho - tl.b0 * d0) * tl.inv_b1 - tl.d2[s];
    }
    const T m = a * d;
    const T v = (T)f + r;
    const T c = (T)lane_c;
    const T xi = v + c;
    const T zeta = tl.K[s] + c * v + (T)0.5 * c * c;
    R += m;
    P += m * xi;
    En += m * zeta;
    if constexpr (SP) X += m * tl.chi[s];
}

// Lane l of the 1-D set: 0 rest (d0), 1/2 +-c1 (d1), 3/4 +-c2 (d2).
__device__ __forceinline__ constexpr int lane_level1(int l) { return l == 0 ? 0 : (l <= 2 ? 1 : 2); }
__device__ __forceinline__ constexpr int lane_sign1(int l) { return l == 0 ? 0 : ((l & 1) ? 1 : -1); }

template <typename T, int H, int TPB, int J, int C1, bool SP, int NF>
__device__ __forceinline__ void gather1_uniform(const Tile1<T>& tl, int f, int64_t x0, int64_t nx,
                                                T* __restrict__ Yn, double (&acc)[NF])
{
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int t = j * TPB + (int)threadIdx.x;
        const int base = t + H - f;  // source of displacement f + o is base - o
        T R = 0, P = 0, En = 0, X = 0;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
#pragma unroll
            for (int l = 0; l < 5; ++l) {
                const int lev = lane_level1(l);
                const int c = lane_sign1(l) * (lev == 0 ? 0 : C1 + lev - 1);
                add_packet1<T, SP>(tl, base - (k + c), f, k, c, lev, R, P, En, X);
            }
        }
        const int64_t x = x0 + t;
        if (x < nx) {
            Yn[x] = R;
            Yn[nx + x] = P;
            Yn[2 * nx + x] = En;
            acc[0] += (double)R;
            acc[1] += (double)P;
            acc[2] += (double)En;
            if constexpr (SP) {
                Yn[3 * nx + x] = X;
                acc[3] += (double)X;
            }
        }
    }
}

template <typename T, int H, int TPB, int J, bool SP, int NF>
__device__ void gather1_general(const Tile1<T>& tl, const TileInfo& ti, int64_t x0, int64_t nx,
                                T* __restrict__ Yn, double (&acc)[NF])
{
    for (int j = 0; j < J; ++j) {
        const int t = j * TPB + (int)threadIdx.x;
        T R = 0, P = 0, En = 0, X = 0;
        for (int k = 0; k < 2; ++k) {
            for (int l = 0; l < 5; ++l) {
                const int lev = lane_level1(l), sg = lane_sign1(l);
                int clo = 0, chi = 0;
                if (lev > 0) {
                    const int a = ti.cmin + lev - 1, b = ti.cmax + lev - 1;
                    clo = sg > 0 ? a : -b;
                    chi = sg > 0 ? b : -a;
                }
                const int lo = max(-H, ti.fxmin + k + clo), hi = min(H, ti.fxmax + k + chi);
                for (int dl = lo; dl <= hi; ++dl) {
                    const int s = t + H - dl;
                    const int p = tl.pk[s];
                    const int fs = lane_fx(p);
                    const int cs = lev == 0 ? 0 : sg * (lane_c1(p) + lev - 1);
                    if (fs + k + cs != dl) continue;
                    add_packet1<T, SP>(tl, s, fs, k, cs, lev, R, P, En, X);
                }
            }
        }
        const int64_t x = x0 + t;
        if (x < nx) {
            Yn[x] = R;
            Yn[nx + x] = P;
            Yn[2 * nx + x] = En;
            acc[0] += (double)R;
            acc[1] += (double)P;
            acc[2] += (double)En;
            if constexpr (SP) {
                Yn[3 * nx + x] = X;
                acc[3] += (double)X;
            }
        }
    }
}

// One tile of TPB * J destinations starting at x0 of a tube of nx nodes, in
// two phases: tile1d_load reads its sources (plus a halo of H, clamped or
// wrapped) into registers; tile1d_gather stages them in LDS, gathers, writes
// Yn and adds the tile's new moments to acc, returning the tile's integer
// summary.  Splitting them lets a persistent block load its next tile while
// it gathers the current one.  tile1d_gather contains block-wide barriers:
// every thread of the block must call it.  WALLS instances also handle
// reflecting walls (the others keep no per-source mirror state); SP instances
// carry the species moment of two gases as a fourth field.
template <typename T, int H, int TPB, int J, bool WALLS, bool SP>
struct Tile1Src {
    static constexpr int W = TPB * J + 2 * H;
    static constexpr int NS = (W + TPB - 1) / TPB;
    static constexpr int NF = SP ? 4 : 3;
    T ld[NS][NF];
    bool mir[WALLS ? NS : 1];  // mirror image beyond a reflecting wall: momentum negated when used
};

template <typename T, int H, int TPB, int J, bool WALLS, bool SP>
__device__ __forceinline__ void tile1d_load(const T* __restrict__ Y, int64_t nx, int bc, int64_t x0,
                                            Tile1Src<T, H, TPB, J, WALLS, SP>& src)
{
    using S = Tile1Src<T, H, TPB, J, WALLS, SP>;
#pragma unroll
    for (int u = 0; u < S::NS; ++u) {
        const int i = (int)threadIdx.x + u * TPB;
        if (i < S::W) {
            const int64_t gx = x0 - H + i;
            int64_t si;
            if constexpr (WALLS) si = source_idx(gx, nx, bc, &src.mir[u]);
            else si = bc == kBcPeriodic ? wrap_near(gx, nx) : clamp_idx(gx, nx);
            src.ld[u][0] = Y[si];
            src.ld[u][1] = Y[nx + si];
            src.ld[u][2] = Y[2 * nx + si];
            if constexpr (SP) src.ld[u][3] = Y[3 * nx + si];
        }
    }
}

template <typename T, int H, int TPB, int J, bool WALLS, bool SP>
__device__ __forceinline__ TileInfo tile1d_gather(const Tile1Src<T, H, TPB, J, WALLS, SP>& src, T* __restrict__ Yn,
                                                  int64_t nx, int64_t x0, const Consts& k,
                                                  double (&acc)[Tile1Src<T, H, TPB, J, WALLS, SP>::NF])
{
    using S = Tile1Src<T, H, TPB, J, WALLS, SP>;
    constexpr int NF = S::NF;
    constexpr int W = S::W;
    constexpr int NW = TPB / 64;
    __shared__ int s_pk[W];
    __shared__ T s_r[W], s_rho[W], s_d2[W], s_K[W];
    __shared__ T s_chi[SP ? W : 1];
    __shared__ int s_red[NW][8];

    TileInfo ti = {INT_MAX, INT_MIN, 0, 0, INT_MAX, INT_MIN, 0, 0};
#pragma unroll
    for (int u = 0; u < S::NS; ++u) {
        const int i = (int)threadIdx.x + u * TPB;
        if (i >= W) break;
        // (the sign of a mirror image is applied here, once its load has
        // arrived, so that loads issued ahead of time are not waited for)
        T mom = src.ld[u][1];
        if constexpr (WALLS) mom = src.mir[u] ? -mom : mom;
        Src1<T> s;
        if constexpr (SP) s = make_src1<T, true>(src.ld[u][0], mom, src.ld[u][2], k, src.ld[u][3]);
        else s = make_src1<T, false>(src.ld[u][0], mom, src.ld[u][2], k);
        if constexpr (SP) s_chi[i] = s.chi;
        s_pk[i] = pack_lane(s.f, 0, s.c1);
        s_r[i] = s.r;
        s_rho[i] = s.bad ? (T)0 : src.ld[u][0];
        s_d2[i] = s.d2;
        s_K[i] = s.K;
        ti.fxmin = min(ti.fxmin, s.f);
        ti.fxmax = max(ti.fxmax, s.f);
        ti.cmin = min(ti.cmin, s.c1);
        ti.cmax = max(ti.cmax, s.c1);
        ti.reach = max(ti.reach, axis_reach(s.f, s.c1));
        ti.bad |= s.bad ? 1 : 0;
    }
    ti = block_tile_info<NW>(ti, s_red);  // contains the barrier after staging
    const Tile1<T> tl = {s_pk, s_r, s_rho, s_d2, s_K, s_chi, (T)k.delta0, (T)k.b0, (T)k.inv_b1};
    const bool uniform = ti.fxmin == ti.fxmax && ti.cmin == ti.cmax && ti.reach <= H;
    if (uniform && ti.cmin == 0)
        gather1_uniform<T, H, TPB, J, 0, SP, NF>(tl, ti.fxmin, x0, nx, Yn, acc);
    else if (uniform && ti.cmin == 1)
        gather1_uniform<T, H, TPB, J, 1, SP, NF>(tl, ti.fxmin, x0, nx, Yn, acc);
    else if (uniform && ti.cmin == 2)
        gather1_uniform<T, H, TPB, J, 2, SP, NF>(tl, ti.fxmin, x0, nx, Yn, acc);
    else if (uniform && ti.cmin == 3)
        gather1_uniform<T, H, TPB, J, 3, SP, NF>(tl, ti.fxmin, x0, nx, Yn, acc);
    else
        gather1_general<T, H, TPB, J, SP, NF>(tl, ti, x0, nx, Yn, acc);
    return ti;
}

template <typename T, int H, int TPB, int J, bool WALLS, bool SP>
__global__ void __launch_bounds__(TPB)
step1d_kernel(const T* __restrict__ Y, T* __restrict__ Yn, Grid g, Consts k,
              StepCtl* __restrict__ ctl, double* __restrict__ partials, long long step)
{
    if (ctl->err_step < step) return;  // an earlier step failed: keep its input intact
    const int64_t x0 = (int64_t)blockIdx.x * (TPB * J);
    using S = Tile1Src<T, H, TPB, J, WALLS, SP>;
    S src;
    tile1d_load<T, H, TPB, J, WALLS, SP>(Y, g.nx, g.bc_x, x0, src);
    double acc[S::NF] = {};
    const TileInfo ti = tile1d_gather<T, H, TPB, J, WALLS, SP>(src, Yn, g.nx, x0, k, acc);
    finish_step<TPB / 64, S::NF>(acc, ti, partials + (int64_t)blockIdx.x * kPartialStride, H);
}

// Pool form: one block per tile of the tile table (1-D tiles cost about the
// same, so the hardware's block scheduling balances them and overlaps one
// tile's loads with other tiles' work).  A tile belongs to one slot; its word
// says whether the slot still steps and which moment set holds its state.
template <typename T, int TPB, int J, bool WALLS, bool SP>
__global__ void __launch_bounds__(TPB) pool1d_kernel(PoolView v, Consts k)
{
    const int t = blockIdx.x;
    if (t >= *v.ntiles) return;
    const int ts = v.tstate[t];
    if (!(ts & kTileLive)) return;  // the same for the whole block
    T* arena = (T*)v.arena;
    const PoolTile& tl = v.tiles[t];
    const int64_t o0 = tl.off[0], o1 = tl.off[1];  // selected below, not indexed (keeps them in registers)
    const int64_t from = (ts & kTileSet) ? o1 : o0, to = (ts & kTileSet) ? o0 : o1;
    const int64_t nx = tl.nx, x0 = tl.x0;
    using S = Tile1Src<T, kHalo, TPB, J, WALLS, SP>;
    S src;
    tile1d_load<T, kHalo, TPB, J, WALLS, SP>(arena + from, nx, tl.bc_x, x0, src);
    double acc[S::NF] = {};
    const TileInfo ti = tile1d_gather<T, kHalo, TPB, J, WALLS, SP>(src, arena + to, nx, x0, k, acc);
    finish_step<TPB / 64, S::NF>(acc, ti, v.partials + (int64_t)t * kPartialStride, kHalo);
}

// Per slot (one block each): the same fixed-order reduction as finalize_kernel
// over the slot's tile rows.
__global__ void __launch_bounds__(kFinTPB) pool_finalize_kernel(PoolView v, int commit)
{
    __shared__ double s_sum[kFinTPB / 64][4];
    __shared__ int s_ir[kFinTPB / 64][2];
    const int p = blockIdx.x;
    if (p == 0 && threadIdx.x == 0) {  // the step kernels of this step are done with their counters
        for (int i = 0; i < 5; ++i) v.next[i] = 0;
    }
    const PoolProb& P = v.probs[p];
    PoolState& S = v.state[p];
    if (!P.active || S.done >= P.target || S.err_step != 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    int reach = 0, err = 0;
    for (int64_t b = P.t0 + tid; b < P.t1; b += kFinTPB) {
        const double* q = v.partials + b * kPartialStride;
#pragma unroll
        for (int f = 0; f < 4; ++f) s[f] += q[f];
        reach = max(reach, (int)q[4]);
        err |= (int)q[5];
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) s[f] = wave_sum(s[f]);
    reach = wave_max(reach);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) err |= __shfl_xor(err, o, 64);
    if (lane == 0) {
#pragma unroll
        for (int f = 0; f < 4; ++f) s_sum[wid][f] = s[f];
        s_ir[wid][0] = reach;
        s_ir[wid][1] = err;
    }
    __shared__ int s_word;
    __syncthreads();
    if (tid == 0 && commit) {
        const int64_t step = S.done + 1;
        for (int f = 0; f < 4; ++f) {
            double t = s_sum[0][f];
            for (int w = 1; w < kFinTPB / 64; ++w) t += s_sum[w][f];
            S.totals[f] = t;
        }
        int r = s_ir[0][0], e = s_ir[0][1];
        for (int w = 1; w < kFinTPB / 64; ++w) { r = max(r, s_ir[w][0]); e |= s_ir[w][1]; }
        S.max_reach = r;
        S.totals_step = step;
        if (e) {
            S.err_code = e;
            S.err_step = step;
        } else {
            S.done = step;
        }
        s_word = (int)(S.done & 1) | (!e && S.done < P.target ? kTileLive : 0);
    }
    __syncthreads();
    if (commit)
        for (int64_t t = P.t0 + tid; t < P.t1; t += kFinTPB) v.tstate[t] = s_word;
}

#ifndef LB_T1_TPB
#define LB_T1_TPB 256
#endif
#ifndef LB_T1_J
#define LB_T1_J 4
#endif
constexpr int k1TPB = LB_T1_TPB, k1J = LB_T1_J;

}  // namespace

int64_t step_blocks_1d(const Grid& g)
{
    const int64_t tile = (int64_t)k1TPB * k1J;
    return (g.nx + tile - 1) / tile;
}

template <typename T>
hipError_t launch_step1d(const T* Y, T* Yn, const Grid& g, const Consts& k, StepCtl* ctl,
                         double* partials, long long step, hipStream_t stream)
{
    const dim3 grid((unsigned)step_blocks_1d(g));
    const bool walls = g.bc_x == kBcReflecting;
    if (k.species) {
        if (walls)
            step1d_kernel<T, kHalo, k1TPB, k1J, true, true><<<grid, k1TPB, 0, stream>>>(Y, Yn, g, k, ctl, partials, step);
        else
            step1d_kernel<T, kHalo, k1TPB, k1J, false, true><<<grid, k1TPB, 0, stream>>>(Y, Yn, g, k, ctl, partials, step);
    } else if (walls) {
        step1d_kernel<T, kHalo, k1TPB, k1J, true, false><<<grid, k1TPB, 0, stream>>>(Y, Yn, g, k, ctl, partials, step);
    } else {
        step1d_kernel<T, kHalo, k1TPB, k1J, false, false><<<grid, k1TPB, 0, stream>>>(Y, Yn, g, k, ctl, partials, step);
    }
    return hipGetLastError();
}

template <typename T, int S>
static hipError_t pool1d_launch_shape(const PoolView& v, const Consts& k, int nblocks, bool walls,
                                      hipStream_t stream)
{
    constexpr int TPB = kPool1TPB[S], J = kPool1J[S];
    if (k.species) {  // two gases: the instances that carry rho chi
        if (walls) pool1d_kernel<T, TPB, J, true, true><<<nblocks, TPB, 0, stream>>>(v, k);
        else pool1d_kernel<T, TPB, J, false, true><<<nblocks, TPB, 0, stream>>>(v, k);
    } else if (walls) {
        pool1d_kernel<T, TPB, J, true, false><<<nblocks, TPB, 0, stream>>>(v, k);
    } else {
        pool1d_kernel<T, TPB, J, false, false><<<nblocks, TPB, 0, stream>>>(v, k);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pool1d(const PoolView& v, const Consts& k, int shape, int nblocks, bool walls,
                         hipStream_t stream)
{
    switch (shape) {
        case 0: return pool1d_launch_shape<T, 0>(v, k, nblocks, walls, stream);
        case 1: return pool1d_launch_shape<T, 1>(v, k, nblocks, walls, stream);
        case 2: return pool1d_launch_shape<T, 2>(v, k, nblocks, walls, stream);
        case 3: return pool1d_launch_shape<T, 3>(v, k, nblocks, walls, stream);
        case 4: return pool1d_launch_shape<T, 4>(v, k, nblocks, walls, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pool_finalize(const PoolView& v, int nslots, int commit, hipStream_t stream)
{
    pool_finalize_kernel<<<nslots, kFinTPB, 0, stream>>>(v, commit);
    return hipGetLastError();
}

hipError_t launch_finalize(double* partials, int64_t nb, StepCtl* ctl, long long step,
                           hipStream_t stream, bool species2d)
{
    if (nb > 16 * kChunk) {  // many rows: fold each chunk first, on many CUs
        const int64_t g = (nb + kChunk - 1) / kChunk;
        partials_chunk_kernel<<<(unsigned)g, kChunk, 0, stream>>>(partials, nb, ctl, step);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        finalize_kernel<<<1, kFinTPB, 0, stream>>>(partials, g, kChunk, ctl, step, species2d ? 1 : 0);
        return hipGetLastError();
    }
    finalize_kernel<<<1, kFinTPB, 0, stream>>>(partials, nb, 1, ctl, step, species2d ? 1 : 0);
    return hipGetLastError();
}

template hipError_t launch_step1d<double>(const double*, double*, const Grid&, const Consts&,
                                          StepCtl*, double*, long long, hipStream_t);
template hipError_t launch_step1d<float>(const float*, float*, const Grid&, const Consts&,
                                         StepCtl*, double*, long long, hipStream_t);

template hipError_t launch_pool1d<double>(const PoolView&, const Consts&, int, int, bool, hipStream_t);
template hipError_t launch_pool1d<float>(const PoolView&, const Consts&, int, int, bool, hipStream_t);

}  // namespace lbsd
