// Device-side building blocks of the tau = 1 semi-discrete LB step on gfx950.
//
// One node's equilibrium (Sec. III.B of Komeili, Mirzaei, Shabouei,
// arXiv 1602.02675) is reduced to the handful of numbers a destination needs
// to rebuild every packet the node emits:
//   f      floor of the flow velocity per axis (corner 0 of eq. 28/29)
//   r      v - f per axis: the interpolation fraction (alpha_1 = r, alpha_0 = 1 - r)
//   c1     c'_1 of eq. 26 (c'_2 = c1 + 1)
//   d0..d2 level weights (eq. 24-25 and d_0 = delta0 rho)
//   K      |v|^2 / 2 + phi, so that a packet on lane c' carries
//          zeta = K + c'.v + |c'|^2 / 2 (eq. 14, 21)
// The integer decisions (f, c1) are taken in the same precision and with the
// same expression order as the plain definition, with FMA contraction off, so
// that the destination of every packet is reproducible bit for bit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbsd {

constexpr int kMaxC1 = 1000;  // caps A (any real reach check fails far earlier)

// Boundary of a grid axis (the values of LB_BC_*).
constexpr int kBcTransmissive = 0;
constexpr int kBcPeriodic = 1;
constexpr int kBcReflecting = 2;

// Problem constants shared by every kernel (lattice units).
struct Consts {
    double Dg1;       // D (gamma - 1)
    double phi_coef;  // 1 - (D/2)(gamma - 1), eq. 15
    double delta0;    // d_0 / rho on the triple-level sets (0 on the square dual-level set)
    double b0;        // rest-lane multiplicity b_0 (1 with a rest level, else 0)
    double inv_b1;    // 1 / b_1
    double rest_q;    // square lattice with a rest level: d_0 / (d_1 + d_2) = b_1 delta0 / (1 - delta0)
    double g1m1;      // two gases: gamma_1 - 1 (gas 1, the species field's gas)
    double g2m1;      // two gases: gamma_2 - 1
    int species;      // 1: two gases, a species moment rho chi after rho E
    int hex;          // 1: the hexagonal lattice (2-D)
};

template <typename T>
struct Src1 {   // one source node of the 1-D lattice
    int f, c1;
    T r, d0, d1, d2, K;
    T chi;      // two gases: mass fraction of gas 1 (what each packet carries per unit mass)
    bool bad;   // rho <= 0 or a non-finite moment
};

template <typename T>
struct Src2 {   // one source node of the square lattice, as the gather uses it
    int fx, fy, c1;
    T vx, ry;     // v_x (lattice units) and the y fraction r_y = v_y - floor(v_y)
    T m[2][2];    // packet mass of level l + 1 (speed c'_{l+1}) at x corner k: d (1 - r_x), d r_x
    T kk[2];      // K + c'^2 / 2 for c' = c'_1, c'_2, with K = |v|^2 / 2 + phi
    T chi;        // two gases: mass fraction of gas 1
    bool bad;
};

// Largest integer c with c*c <= A, for 0 <= A <= kMaxC1^2 (eq. 26: "int" of sqrt).
template <typename T>
__device__ __forceinline__ int isqrt_floor(T A)
{
#pragma clang fp contract(off)
    // a single-precision root is within one of floor(sqrt(A)) for the clamped
    // A <= kMaxC1^2 (relative error < 1e-7); the exact comparisons settle it
    int c = (int)sqrtf((float)A);
    if (c > 0 && (T)c * (T)c > A) --c;
    if ((T)(c + 1) * (T)(c + 1) <= A) ++c;
    return c;
}

// a / b in the per-node primitives.  FAST = false (FP64 storage): the
// correctly rounded quotient, so that floor(v) and c'_1 match the plain
// definition bit for bit.  FAST = true (FP32 storage, whose results are
// rounded to FP32 and whose decisions the step does not need bit for bit):
// the hardware reciprocal refined by one Newton step, r (2 - b r), in two
// FMAs, then a product; relative error near 1e-16, far below FP32 rounding,
// for a few instructions instead of the IEEE division sequence.  b > 0, finite.
template <bool FAST>
__device__ __forceinline__ double pdiv(double a, double b)
{
    if constexpr (FAST) {
        double r = __builtin_amdgcn_rcp(b);
        r = __builtin_fma(r, __builtin_fma(-b, r, 1.0), r);
        return a * r;
    } else {
#pragma clang fp contract(off)
        return a / b;
    }
}

// Internal energy, c'_1 and the weight split of one node.  rho > 0 required.
//  e = E - |v|^2/2 (clamped at 0), A = D(gamma-1) e rho / (rho - b0 d0),
//  c1 = floor(sqrt(A)); with w = (A - c1^2) / (c2^2 - c1^2) in [0, 1):
//  b1 d2 = (rho - b0 d0) w and b1 d1 = (rho - b0 d0)(1 - w), which is eq. 24-25
//  rewritten (both sum to rho - b0 d0 and satisfy sum b d c'^2 = D p).
template <typename T>
struct Levels {
    T e, A, rest;
    int c1;
};

template <typename T, bool FAST = false>
__device__ __forceinline__ Levels<T> node_levels(T rho, T v2, T E, T d0, const Consts& k)
{
#pragma clang fp contract(off)
    Levels<T> L;
    T e = E - (T)0.5 * v2;
    if (e < (T)0) e = (T)0;
    L.e = e;
    L.rest = rho - (T)k.b0 * d0;
    T A = pdiv<FAST>((T)k.Dg1 * e * rho, L.rest);
    if (!(A >= (T)0)) A = (T)0;
    if (A > (T)kMaxC1 * (T)kMaxC1) A = (T)kMaxC1 * (T)kMaxC1;
    L.A = A;
    L.c1 = isqrt_floor<T>(A);
    return L;
}

template <typename T>
__device__ __forceinline__ bool finite_val(T x) { return isfinite(x); }

// w = (A - c'_1^2) / (2 c'_1 + 1) in [0, 1]: the share of level 2 (eq. 24-25
// rewritten; b_1 d_2 = (rho - b_0 d_0) w).  The divisor is a small odd
// integer: its reciprocal is a constant for the usual c'_1 <= 3.
__device__ __forceinline__ double level_w(double A, int c1)
{
    const double num = A - (double)(c1 * c1);
    double w;
    if (c1 <= 3)
        w = num * (c1 == 0 ? 1.0 : (c1 == 1 ? 1.0 / 3.0 : (c1 == 2 ? 1.0 / 5.0 : 1.0 / 7.0)));
    else
        w = num / (double)(2 * c1 + 1);
    return w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
}

// Per-node primitives, level speeds, weights and interpolation split of one
// source (eq. 15, 24-26, 28-29).  They are computed in FP64 whatever the
// storage type T: in FP32 storage the per-node energy bookkeeping (E -> e, A,
// the d_1 / d_2 split near a switch of c'_1) is where FP32 arithmetic would
// lose the most, and FP64 costs the same VALU issue rate on this chip (FP32
// storage takes its quotients from a refined reciprocal, see pdiv).  The
// staged results are rounded to T.  SP: two gases; m3t is the species moment
// rho chi, and the node's gas is the mixture of the two by mass fraction
// (c_v weighted, one gas constant): gamma - 1 = 1 / (chi / (gamma_1 - 1) +
// (1 - chi) / (gamma_2 - 1)), which sets phi (eq. 15) and A (eq. 26).
template <typename T, bool SP = false>
__device__ __forceinline__ Src1<T> make_src1(T m0t, T m1t, T m2t, const Consts& kc, T m3t = (T)0)
{
    const double m0 = m0t, m1 = m1t, m2 = m2t;
    Src1<T> s;
    s.bad = !(m0 > 0.0) || !finite_val(m0) || !finite_val(m1) || !finite_val(m2) ||
            (SP && !finite_val((double)m3t));
    s.chi = (T)0;
    if (s.bad) {
        s.f = 0; s.c1 = 0;
        s.r = (T)0; s.d0 = (T)0; s.d1 = (T)0; s.d2 = (T)0; s.K = (T)0;
        return s;
    }
    Consts k = kc;
    constexpr bool FAST = sizeof(T) < 8;
    if constexpr (SP) {
#pragma clang fp contract(off)
        double chi = pdiv<FAST>((double)m3t, m0);
        chi = chi < 0.0 ? 0.0 : (chi > 1.0 ? 1.0 : chi);
        const double gm1 = pdiv<FAST>(1.0, pdiv<FAST>(chi, k.g1m1) + pdiv<FAST>(1.0 - chi, k.g2m1));
        k.Dg1 = 1.0 * gm1;
        k.phi_coef = 1.0 - 0.5 * gm1;
        s.chi = (T)chi;
    }
    double v, E, v2, d0;
    {
#pragma clang fp contract(off)
        v = pdiv<FAST>(m1, m0);
        E = pdiv<FAST>(m2, m0);
        v2 = v * v;
        d0 = k.delta0 * m0;
    }
    Levels<double> L = node_levels<double, FAST>(m0, v2, E, d0, k);
    const double fv = floor(v);
    s.f = (int)fv;
    s.r = (T)(v - fv);
    s.c1 = L.c1;
    const double per = L.rest * k.inv_b1;
    const double d2 = per * level_w(L.A, L.c1);
    s.d2 = (T)d2;
    s.d1 = (T)(per - d2);
    s.d0 = (T)d0;
    s.K = (T)(0.5 * v2 + k.phi_coef * L.e);
    return s;
}

// REST: the square set with a rest level (d_0 = delta0 rho); the staged level
// masses then carry (rho - d_0) / b_1 between them.  SP: two gases; m4t is
// the species moment rho chi and the node's gas the mixture (as in make_src1,
// with D = 2).  VY0: for callers that use the result only where rho v_y is
// +-0: v_y is then taken as rho v_y itself, the same +-0 as the quotient
// (elsewhere v_y = rho v_y, and floor(v_y) and r_y tell that it is not 0).
template <typename T, bool REST = false, bool SP = false, bool VY0 = false>
__device__ __forceinline__ Src2<T> make_src2(T m0t, T m1t, T m2t, T m3t, const Consts& kc, T m4t = (T)0)
{
    const double m0 = m0t, m1 = m1t, m2 = m2t, m3 = m3t;
    Src2<T> s;
    s.bad = !(m0 > 0.0) || !finite_val(m0) || !finite_val(m1) || !finite_val(m2) || !finite_val(m3) ||
            (SP && !finite_val((double)m4t));
    s.chi = (T)0;
    Consts k = kc;
    constexpr bool FAST = sizeof(T) < 8;
    if constexpr (SP) {
#pragma clang fp contract(off)
        double chi = pdiv<FAST>((double)m4t, m0 > 0.0 ? m0 : 1.0);
        chi = chi < 0.0 ? 0.0 : (chi > 1.0 ? 1.0 : chi);
        const double gm1 = pdiv<FAST>(1.0, pdiv<FAST>(chi, k.g1m1) + pdiv<FAST>(1.0 - chi, k.g2m1));
        k.Dg1 = 2.0 * gm1;
        k.phi_coef = 1.0 - 1.0 * gm1;
        s.chi = (T)chi;
    }
    if (s.bad) {
        s.fx = 0; s.fy = 0; s.c1 = 0;
        s.vx = (T)0; s.ry = (T)0;
        s.m[0][0] = s.m[0][1] = s.m[1][0] = s.m[1][1] = (T)0;
        s.kk[0] = s.kk[1] = (T)0;
        return s;
    }
    double vx, vy, E, v2;
    {
#pragma clang fp contract(off)
        vx = pdiv<FAST>(m1, m0);
        vy = VY0 ? m2 : pdiv<FAST>(m2, m0);
        E = pdiv<FAST>(m3, m0);
        v2 = vx * vx + vy * vy;
    }
    Levels<double> L = node_levels<double, FAST>(m0, v2, E, REST ? k.delta0 * m0 : 0.0, k);
    const double fvx = floor(vx), fvy = floor(vy);
    s.fx = (int)fvx;
    s.fy = (int)fvy;
    const double rx = vx - fvx;
    s.vx = (T)vx;
    s.ry = (T)(vy - fvy);
    s.c1 = L.c1;
    const double d2 = L.rest * k.inv_b1 * level_w(L.A, L.c1);
    const double d1 = L.rest * k.inv_b1 - d2;
    s.m[0][0] = (T)(d1 * (1.0 - rx));
    s.m[0][1] = (T)(d1 * rx);
    s.m[1][0] = (T)(d2 * (1.0 - rx));
    s.m[1][1] = (T)(d2 * rx);
    const double K = 0.5 * v2 + k.phi_coef * L.e;
    const double c1 = (double)L.c1;
    s.kk[0] = (T)(K + 0.5 * c1 * c1);
    s.kk[1] = (T)(K + 0.5 * (c1 + 1.0) * (c1 + 1.0));
    return s;
}

template <typename T>
struct SrcHex {   // one source node of the hexagonal lattice
    int fa, fb;   // floor of the axial coordinates (a, b) of v = a e_1 + b e_2
    int c1;
    int tri;      // triangle of the cell that holds the end point of v: 0 has
                  // the vertex (0, 0), 1 the vertex (1, 1) (both (1,0), (0,1))
    T ra, rb;     // (a, b) - (f_a, f_b)
    T vx, vy;     // Cartesian v (lattice units)
    T K;          // |v|^2 / 2 + phi
    T d0, d1, d2; // level weights (d0 = 0 without the rest group)
    bool bad;
};

constexpr double kSqrt3 = 1.7320508075688772;  // sqrt(3), correctly rounded

// Per-node primitives of a source of the hexagonal lattice (Fig. 1; eq. 15,
// 24-26 with b_1 = b_2 = 6, Consts::inv_b1 = 1/6): as make_src2, and the end
// point of v in axial coordinates, b = 2 v_y / sqrt(3), a = v_x - b / 2 (e_1 =
// (1, 0), e_2 = (1/2, sqrt(3)/2)), whose cell (f_a, f_b) + [0, 1]^2 splits
// into the triangles below and above the diagonal r_a + r_b = 1.  REST: the
// set with a rest group, d_0 = delta0 rho.
template <typename T, bool REST>
__device__ __forceinline__ SrcHex<T> make_srchex(T m0t, T m1t, T m2t, T m3t, const Consts& k)
{
    const double m0 = m0t, m1 = m1t, m2 = m2t, m3 = m3t;
    SrcHex<T> s;
    s.bad = !(m0 > 0.0) || !finite_val(m0) || !finite_val(m1) || !finite_val(m2) || !finite_val(m3);
    if (s.bad) {
        s.fa = 0; s.fb = 0; s.c1 = 0; s.tri = 0;
        s.ra = s.rb = s.vx = s.vy = s.K = s.d0 = s.d1 = s.d2 = (T)0;
        return s;
    }
    constexpr bool FAST = sizeof(T) < 8;
    double vx, vy, E, v2, a, b;
    {
#pragma clang fp contract(off)
        vx = pdiv<FAST>(m1, m0);
        vy = pdiv<FAST>(m2, m0);
        E = pdiv<FAST>(m3, m0);
        v2 = vx * vx + vy * vy;
        b = pdiv<FAST>(2.0 * vy, kSqrt3);
        a = vx - 0.5 * b;
    }
    const double d0 = REST ? k.delta0 * m0 : 0.0;
    Levels<double> L = node_levels<double, FAST>(m0, v2, E, d0, k);
    // floors clamped far beyond any admissible reach (the step reports those)
    const double fa = fmin(fmax(floor(a), -32.0), 31.0), fb = fmin(fmax(floor(b), -32.0), 31.0);
    s.fa = (int)fa;
    s.fb = (int)fb;
    const double ra = a - fa, rb = b - fb;
    s.tri = ra + rb > 1.0 ? 1 : 0;
    s.ra = (T)ra;
    s.rb = (T)rb;
    s.vx = (T)vx;
    s.vy = (T)vy;
    s.c1 = L.c1;
    const double per = L.rest * k.inv_b1;
    const double d2 = per * level_w(L.A, L.c1);
    s.d2 = (T)d2;
    s.d1 = (T)(per - d2);
    s.d0 = (T)d0;
    s.K = (T)(0.5 * v2 + k.phi_coef * L.e);
    return s;
}

// Reach of a node: the largest |displacement| of any of its packets along one
// axis, max(f + 1 + c'_2, c'_2 - f).
__device__ __forceinline__ int axis_reach(int f, int c1)
{
    const int c2 = c1 + 1;
    const int a = f + 1 + c2, b = c2 - f;
    return a > b ? a : b;
}

// Wavefront (64-lane) reductions.
template <typename V>
__device__ __forceinline__ V wave_sum(V x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}
__device__ __forceinline__ int wave_max(int x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) { int y = __shfl_xor(x, o, 64); x = y > x ? y : x; }
    return x;
}
__device__ __forceinline__ int wave_min(int x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) { int y = __shfl_xor(x, o, 64); x = y < x ? y : x; }
    return x;
}

__device__ __forceinline__ int64_t wrap_idx(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}
// Periodic index for i within a few periods of [0, n): the full modulo runs
// only for the (halo) indices that are out of range.
__device__ __forceinline__ int64_t wrap_near(int64_t i, int64_t n)
{
    if (i >= 0 && i < n) return i;
    if (i < 0 && i + n >= 0) return i + n;
    if (i >= n && i - n < n) return i - n;
    return wrap_idx(i, n);
}
__device__ __forceinline__ int64_t clamp_idx(int64_t i, int64_t n)
{
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}
// Reflecting walls stand on the outer faces of nodes 0 and n - 1: a node
// beyond a wall is the mirror image of node -1 - i (low end) or 2n - 1 - i
// (high end), with its normal momentum negated.  Sources within the halo of
// the domain (n >= halo) map exactly; indices further out, which only the
// spare columns of a last tile read and whose packets reach no destination,
// are clamped into range.
__device__ __forceinline__ int64_t mirror_idx(int64_t i, int64_t n)
{
    if (i < 0) { const int64_t m = -1 - i; return m < n ? m : n - 1; }
    if (i >= n) { const int64_t m = 2 * n - 1 - i; return m >= 0 ? m : 0; }
    return i;
}
// Source index of (possibly halo) index i along an axis of n nodes with
// boundary bc; *mirrored tells whether the normal momentum must be negated.
__device__ __forceinline__ int64_t source_idx(int64_t i, int64_t n, int bc, bool* mirrored)
{
    *mirrored = bc == kBcReflecting && (i < 0 || i >= n);
    if (bc == kBcPeriodic) return wrap_near(i, n);
    if (bc == kBcReflecting) return mirror_idx(i, n);
    return clamp_idx(i, n);
}

// Persistent blocks take tiles from a shared counter in claim order: a slow
// tile (a transition region, a hot problem) then delays only the block that
// holds it.  Which block computes a tile changes no result.  *s_slot is a
// shared-memory int; every thread of the block must call this.
__device__ __forceinline__ int claim_tile(int* counter, int* s_slot)
{
    __syncthreads();  // the previous claim has been read by every thread
    if (threadIdx.x == 0) *s_slot = atomicAdd(counter, 1);
    __syncthreads();
    return *s_slot;
}

}  // namespace lbsd
