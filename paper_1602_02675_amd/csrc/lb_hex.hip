// The tau = 1 step on the hexagonal lattice (Fig. 1 of Komeili, Mirzaei,
// Shabouei, arXiv 1602.02675; Sec. III.B with b_v = 6), as a gather.
//
// Nodes sit at i e_1 + j e_2 (e_1 = (1, 0), e_2 = (1/2, sqrt(3)/2), unit
// spacing), stored SoA Y[f][j][i]; momenta are Cartesian.  A source node
// emits, per lane (rest group; six directions u_d at c'_1 and at c'_2), one
// packet to each vertex of the lattice triangle around the end point of its
// velocity, with the vertex's barycentric weight: mass alpha_k d_v (eq. 23),
// momentum m (v + c' u_d), energy m (K + c' u_d . v + c'^2 / 2) with K =
// |v|^2 / 2 + phi (eq. 14, 21), to x + f + k + c' u_d in axial steps.
//
// One block computes a tile of kHX x kHY destination nodes.  It stages the
// per-node records (make_srchex) of the tile and a halo of H = kHalo nodes
// along both axial directions in LDS, then each thread sums, for its
// destination, every packet that lands there: it walks the lanes and, per
// lane, the packet classes (floor of the axial velocity, triangle vertex) the
// block's sources can have, and takes a class from the one source that would
// emit it, if that source has the class's floor, speed and triangle.  The
// order of the sum is fixed (deterministic results), and a window of uniform
// floors and speeds costs four candidates per lane.
#include "lb_kernels.hpp"

namespace lbsd {
namespace {

constexpr int kHX = 64, kHY = 16, kHH = kHalo;  // tile (axial i x j) and halo
constexpr int kHTPB = kHX * kHY;                // one destination per thread
constexpr int kSW = kHX + 2 * kHH, kSH = kHY + 2 * kHH, kSN = kSW * kSH;  // staged sources
constexpr int kHNW = kHTPB / 64;

// The six directions: axial steps (DA, DB) and Cartesian unit vectors (UX, UY).
__device__ constexpr int kDA[6] = {1, 0, -1, -1, 0, 1};
__device__ constexpr int kDB[6] = {0, 1, 1, 0, -1, -1};
constexpr double kH3 = 0.8660254037844386;  // sqrt(3) / 2, correctly rounded
__device__ constexpr double kUX[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
__device__ constexpr double kUY[6] = {0.0, kH3, kH3, 0.0, -kH3, -kH3};

// Staged record key: f_a + 64 (bits 0-6), f_b + 64 (7-13), c'_1 (14-23),
// triangle (24); bit 25 marks a bad source (which emits nothing).
__device__ __forceinline__ int hkey(int fa, int fb, int c1) { return (fa + 64) | ((fb + 64) << 7) | (c1 << 14); }
__device__ __forceinline__ int hk_fa(int p) { return (p & 127) - 64; }
__device__ __forceinline__ int hk_fb(int p) { return ((p >> 7) & 127) - 64; }
__device__ __forceinline__ int hk_c1(int p) { return (p >> 14) & 1023; }
constexpr int kHkTri = 1 << 24, kHkBad = 1 << 25;
constexpr int kHkC1 = 1023 << 14;

__device__ __forceinline__ double hfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float hfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Staged records.  w[t]: barycentric weight of vertex t of the source's
// triangle: t = 0 the vertex (0,0) or (1,1) (by the triangle), t = 1 (1,0),
// t = 2 (0,1).
template <typename T, bool REST>
struct HexStage {
    int pk[kSN];
    T vx[kSN], vy[kSN], K[kSN], d1[kSN], d2[kSN];
    T w[3][kSN];
    T d0[REST ? kSN : 1];
};

template <typename T, bool REST>
__global__ void __launch_bounds__(kHTPB)
hex_step_kernel(const T* __restrict__ Y, T* __restrict__ Yn, Grid g, Consts k, StepCtl* __restrict__ ctl,
                double* __restrict__ partials, long long step)
{
    __shared__ HexStage<T, REST> st;
    __shared__ int s_rng[kHNW][6];
    __shared__ double s_sum[kHNW][4];
    __shared__ int s_ir[kHNW][2];
    if (ctl->err_step < step) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t nx = g.nx, ny = g.ny, nn = nx * ny;
    const int64_t tiles_x = (nx + kHX - 1) / kHX;  // tiles row-major, i fastest
    const int64_t X0 = ((int64_t)blockIdx.x % tiles_x) * kHX, Y0 = ((int64_t)blockIdx.x / tiles_x) * kHY;

    // stage the records of the tile and its halo (boundaries map the halo)
    int falo = 1 << 20, fahi = -(1 << 20), fblo = 1 << 20, fbhi = -(1 << 20), clo = 1 << 20, chi = -1;
    for (int q = tid; q < kSN; q += kHTPB) {
        const int lj = q / kSW, li = q - lj * kSW;
        const int64_t gi = X0 - kHH + li, gj = Y0 - kHH + lj;
        const int64_t si = g.bc_x == kBcPeriodic ? wrap_near(gi, nx) : clamp_idx(gi, nx);
        const int64_t sj = g.bc_y == kBcPeriodic ? wrap_near(gj, ny) : clamp_idx(gj, ny);
        const int64_t p = sj * nx + si;
        const SrcHex<T> s = make_srchex<T, REST>(Y[p], Y[nn + p], Y[2 * nn + p], Y[3 * nn + p], k);
        const int c1 = min(s.c1, 1023);
        st.pk[q] = hkey(s.fa, s.fb, c1) | (s.tri ? kHkTri : 0) | (s.bad ? kHkBad : 0);
        st.vx[q] = s.vx;
        st.vy[q] = s.vy;
        st.K[q] = s.K;
        st.d1[q] = s.d1;
        st.d2[q] = s.d2;
        {
#pragma clang fp contract(off)
            const T ra = s.ra, rb = s.rb;
            st.w[0][q] = s.tri ? (ra + rb) - (T)1 : ((T)1 - ra) - rb;
            st.w[1][q] = s.tri ? (T)1 - rb : ra;
            st.w[2][q] = s.tri ? (T)1 - ra : rb;
        }
        if constexpr (REST) st.d0[q] = s.d0;
        if (!s.bad) {
            falo = min(falo, s.fa); fahi = max(fahi, s.fa);
            fblo = min(fblo, s.fb); fbhi = max(fbhi, s.fb);
            clo = min(clo, c1); chi = max(chi, c1);
        }
    }
    falo = wave_min(falo); fahi = wave_max(fahi);
    fblo = wave_min(fblo); fbhi = wave_max(fbhi);
    clo = wave_min(clo); chi = wave_max(chi);
    if (lane == 0) {
        s_rng[wid][0] = falo; s_rng[wid][1] = fahi; s_rng[wid][2] = fblo;
        s_rng[wid][3] = fbhi; s_rng[wid][4] = clo; s_rng[wid][5] = chi;
    }
    __syncthreads();
    for (int w = 0; w < kHNW; ++w) {
        falo = min(falo, s_rng[w][0]); fahi = max(fahi, s_rng[w][1]);
        fblo = min(fblo, s_rng[w][2]); fbhi = max(fbhi, s_rng[w][3]);
        clo = min(clo, s_rng[w][4]); chi = max(chi, s_rng[w][5]);
    }
    // packets that would move further than the halo are reported (reach),
    // not gathered: the loops stay within it
    falo = max(falo, -kHH - 1); fahi = min(fahi, kHH);
    fblo = max(fblo, -kHH - 1); fbhi = min(fbhi, kHH);
    chi = min(chi, kHH);

    // Gather the packets that land on this thread's destination, lane by
    // lane: for each lane (c', u), sum over its sources m, m v_x, m v_y, m K,
    // then add the lane's packets at once: m (v + c' u) and m (K + c' u . v
    // + c'^2 / 2) (eq. 14, 21).  Within a lane the candidates are taken by
    // floor of the axial velocity and by triangle vertex; the source of a
    // candidate emits it if it has that floor, speed and triangle.
    const int li = tid % kHX, lj = tid / kHX;
    const int cidx = (lj + kHH) * kSW + (li + kHH);  // staged index of the destination node
    double R = 0.0, PX = 0.0, PY = 0.0, E = 0.0;
    // sources of vertex kc at displacement (dx, dy) with key `want` (under
    // `mask`), weight of that vertex times the level weight dl
    auto take = [&](int dx, int dy, int mask, int want, int t, const T* dl, T& s0, T& s1, T& s2, T& s3) {
        if (dx < -kHH || dx > kHH || dy < -kHH || dy > kHH) return;
        const int s = cidx - dy * kSW - dx;
        if ((st.pk[s] & mask) != want) return;
        const T m = st.w[t][s] * dl[s];
        s0 += m;
        s1 = hfma(m, st.vx[s], s1);
        s2 = hfma(m, st.vy[s], s2);
        s3 = hfma(m, st.K[s], s3);
    };
    // the candidates of one lane (speed c, axial step (da, db)); lev: level
    // of the speed (-1: rest group)
    auto lane_sum = [&](int lev, int c, int da, int db, T& s0, T& s1, T& s2, T& s3) {
        const T* dl = lev < 0 ? st.d0 : (lev == 0 ? st.d1 : st.d2);
        const int cmask = lev < 0 ? 0 : kHkC1;  // the rest group moves at any c'_1
        for (int fa = falo; fa <= fahi; ++fa) {
            for (int fb = fblo; fb <= fbhi; ++fb) {
                const int base = hkey(fa, fb, lev < 0 ? 0 : c - lev) & (0x3FFF | cmask);
                const int dx = fa + c * da, dy = fb + c * db;
                // vertex (0,0) of triangle 0, (1,1) of triangle 1, (1,0), (0,1) of either
                take(dx, dy, 0x3FFF | cmask | kHkTri | kHkBad, base, 0, dl, s0, s1, s2, s3);
                take(dx + 1, dy + 1, 0x3FFF | cmask | kHkTri | kHkBad, base | kHkTri, 0, dl, s0, s1, s2, s3);
                take(dx + 1, dy, 0x3FFF | cmask | kHkBad, base, 1, dl, s0, s1, s2, s3);
                take(dx, dy + 1, 0x3FFF | cmask | kHkBad, base, 2, dl, s0, s1, s2, s3);
            }
        }
    };
    if constexpr (REST) {
        T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        lane_sum(-1, 0, 0, 0, s0, s1, s2, s3);
        R += (double)s0;
        PX += (double)s1;
        PY += (double)s2;
        E += (double)s3;
    }
#pragma unroll
    for (int lev = 0; lev < 2; ++lev) {
        for (int c = clo + lev; c <= chi + lev; ++c) {
            if (c > kHH) break;
            const T cc = (T)c, hc2 = (T)0.5 * cc * cc;
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
                lane_sum(lev, c, kDA[d], kDB[d], s0, s1, s2, s3);
                const T cux = cc * (T)kUX[d], cuy = cc * (T)kUY[d];
                R += (double)s0;
                PX += (double)hfma(cux, s0, s1);
                PY += (double)hfma(cuy, s0, s2);
                E += (double)(hfma(hc2, s0, s3) + hfma(cux, s1, cuy * s2));
            }
        }
    }

    // write the destination, and the block's partials
    const int64_t gi = X0 + li, gj = Y0 + lj;
    const bool in = gi < nx && gj < ny;
    int reach = 0, bad = 0;
    if (in) {
        const int64_t q = gj * nx + gi;
        const T r = (T)R, px = (T)PX, py = (T)PY, en = (T)E;
        Yn[q] = r;
        Yn[nn + q] = px;
        Yn[2 * nn + q] = py;
        Yn[3 * nn + q] = en;
        R = r, PX = px, PY = py, E = en;  // the totals are those of the stored fields
        const int p = st.pk[cidx];  // this node as a source
        bad = (p & kHkBad) ? 1 : 0;
        reach = max(axis_reach(hk_fa(p), hk_c1(p)), axis_reach(hk_fb(p), hk_c1(p)));
    } else {
        R = PX = PY = E = 0.0;
    }
    R = wave_sum(R);
    PX = wave_sum(PX);
    PY = wave_sum(PY);
    E = wave_sum(E);
    reach = wave_max(reach);
    bad = wave_max(bad);
    if (lane == 0) {
        s_sum[wid][0] = R; s_sum[wid][1] = PX; s_sum[wid][2] = PY; s_sum[wid][3] = E;
        s_ir[wid][0] = reach;
        s_ir[wid][1] = bad;
    }
    __syncthreads();
    if (tid == 0) {
        double* prow = partials + (int64_t)blockIdx.x * kPartialStride;
        int rr = 0, bb = 0;
        for (int f = 0; f < 4; ++f) {
            double t = s_sum[0][f];
            for (int w = 1; w < kHNW; ++w) t += s_sum[w][f];
            prow[f] = t;
        }
        for (int w = 0; w < kHNW; ++w) {
            rr = max(rr, s_ir[w][0]);
            bb |= s_ir[w][1];
        }
        prow[4] = (double)rr;
        prow[5] = (double)((rr > kHH ? kErrReach : 0) | (bb ? kErrState : 0));
        prow[6] = 0.0;
    }
}

}  // namespace

int64_t hex_blocks(const Grid& g)
{
    return ((g.nx + kHX - 1) / kHX) * ((g.ny + kHY - 1) / kHY);
}

template <typename T>
hipError_t launch_hex(const T* Y, T* Yn, const Grid& g, const Consts& k, StepCtl* ctl, double* partials,
                      long long step, hipStream_t stream)
{
    const unsigned grid = (unsigned)hex_blocks(g);
    if (k.b0 > 0.0)
        hex_step_kernel<T, true><<<grid, kHTPB, 0, stream>>>(Y, Yn, g, k, ctl, partials, step);
    else
        hex_step_kernel<T, false><<<grid, kHTPB, 0, stream>>>(Y, Yn, g, k, ctl, partials, step);
    return hipGetLastError();
}

template hipError_t launch_hex<double>(const double*, double*, const Grid&, const Consts&, StepCtl*, double*,
                                       long long, hipStream_t);
template hipError_t launch_hex<float>(const float*, float*, const Grid&, const Consts&, StepCtl*, double*,
                                      long long, hipStream_t);

}  // namespace lbsd
