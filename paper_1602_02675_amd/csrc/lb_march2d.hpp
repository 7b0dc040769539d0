#pragma once
// Square-lattice step as a column march (Sec. IV.B and V.A of Komeili,
// Mirzaei, Shabouei, arXiv 1602.02675; tau = 1 so a step is the migration of
// the equilibrium, eq. 10 / eq. 30).
//
// Every packet moves along x by floor(v_x) + k_x (+ c' for x-lanes) and along y
// by floor(v_y) + k_y (+ c' for y-lanes).  The kernel splits the two:
//   - a tile is 256 consecutive source columns (the middle 256 - 2H of them
//     are its destination columns) by a strip of destination rows; a block of
//     256 threads marches down the strip (persistent blocks claim tiles);
//   - per source row, each thread turns its node's moments into what its
//     packets need (floor v, r_y, c'_1, v_x, the packet masses per level and
//     x corner, K + c'^2 / 2 per level) once and stages them in an LDS row
//     buffer (double-buffered: one barrier per staged group of rows);
//   - each destination thread gathers the packets that move into its column
//     from the staged row (the x part of the migration) and adds each to a
//     register FIFO of pending destination rows, indexed by the y
//     displacement o = floor(v_y) + k_y (+ c' for y-lanes), o in [-L, L]
//     (the y part); once source row r is in, the FIFO slot of row r - L can
//     receive nothing more and is written out.
// Where the staged sources around a wavefront share floor(v) and c'_1, or
// take two adjacent values of one of floor(v_x) and c'_1 (the integer parts of
// the migration vectors are piecewise constant), the packet classes have
// compile-time column offsets and FIFO slots; elsewhere candidate sources are
// matched at run time.  The same packets are summed either way; only the
// summation order differs from the scatter definition.
//
// The kernels and helpers below sit in an anonymous namespace: each
// translation unit that includes this header instantiates its own kernels
// (lb_march2d.hip and lb_pool2d.hip the one-gas plain and pool forms,
// lb_march2d_sp.hip and lb_pool2d_sp.hip the two-gas ones), and no kernel is
// instantiated in two of them.
#include <climits>

#include "lb_kernels.hpp"

namespace lbsd {

namespace {

constexpr int kMTPB = 256;        // threads (= staged source columns) per block
constexpr int kMNW = kMTPB / 64;  // wavefronts per block
constexpr int kMH = kHalo;        // x halo (largest displacement per axis)
// The FIFO covers y displacements o in [-L, L] (2L + 1 slots).  L = H covers
// every packet; L = 3 covers every source with c'_1 <= 1 and |floor(v_y)|
// small (y-reach <= 3), and leaves registers for two wavefronts per SIMD.
constexpr int kLFull = kMH, kLSmall = 3;
constexpr int kMinRows = 16;      // smallest strip height (bounds the y-halo overhead)

// FIFO values per slot.  The y-momentum is kept as two parts: what packets
// carry as m v_y, and the m c' of the y-lanes (YLaneSum).  A y-lane packet
// and its mirror (opposite sign) reach a destination from two different
// source rows, after other terms; the y-lane sum makes them cancel exactly
// when those rows are equal, so a planar flow keeps v_y = 0 exactly and
// floor(v_y) stays uniform.
enum { kR = 0, kPx = 1, kPyv = 2, kE = 3, kNV = 4 };

// (h, l) += x with the rounding error of h + x carried into l (TwoSum).
template <typename T>
__device__ __forceinline__ void dd_add(T& h, T& l, T x)
{
#pragma clang fp contract(off)
    const T s = h + x;
    const T bp = s - h;
    const T e = (h - (s - bp)) + (x - bp);
    h = s;
    l = l + e;
}

// Sum of the y-lane momenta m c' of one FIFO slot, in double-length
// (TwoSum) arithmetic: FP64 pairs for both storage types.  The terms of one
// destination can span some 80 binades (near rest, a corner weight 1 - r_x
// of 1e-24 next to one of 1), and the row path adds one term per packet
// class; only a double-length sum cancels such mirrored terms from equal rows
// exactly.  In FP32 storage the terms are FP32 products, so an FP64 pair is
// exact where an FP32 pair leaves the rounding of its low part behind.
template <typename T>
struct YLaneSum {
    double h, l;
    __device__ __forceinline__ void zero() { h = l = 0.0; }
    __device__ __forceinline__ void add(T x) { dd_add<double>(h, l, (double)x); }
    __device__ __forceinline__ double total() const { return h + l; }
};

__device__ __forceinline__ int mpack(int fx, int fy, int c1)
{
    fx = fx < -127 ? -127 : (fx > 127 ? 127 : fx);
    fy = fy < -127 ? -127 : (fy > 127 ? 127 : fy);
    c1 = c1 > 255 ? 255 : c1;
    return (fx + 128) | ((fy + 128) << 8) | (c1 << 16);
}
__device__ __forceinline__ int mfx(int p) { return (p & 255) - 128; }
__device__ __forceinline__ int mfy(int p) { return ((p >> 8) & 255) - 128; }
__device__ __forceinline__ int mc1(int p) { return (p >> 16) & 255; }

template <typename T, bool SP>
struct MRowSpecies {  // two gases: mass fraction of gas 1 per source
    T chi[kMTPB];
};
template <typename T>
struct MRowSpecies<T, false> {};  // one gas: empty (the row keeps its layout)

template <typename T, bool RYS>
struct MRowRy {  // the y fraction r_y per source
    T ry[kMTPB];
};
template <typename T>
struct MRowRy<T, false> {};  // rows of the lean pass: every source has v_y = 0 (r_y = 0)

template <typename T, bool SP = false, bool RYS = true>
struct MRow : MRowSpecies<T, SP>, MRowRy<T, RYS> {  // one staged source row (per source, see Src2)
    static constexpr bool kSP = SP, kRYS = RYS;
    using value_type = T;
    T vx[kMTPB];
    T m[2][2][kMTPB];  // [level][x corner]
    T kk[2][kMTPB];    // [level]
    int pk[kMTPB];
};

// chi of the source in column s (0 with one gas)
template <typename Row>
__device__ __forceinline__ typename Row::value_type chi_of(const Row& R, int s)
{
    if constexpr (Row::kSP) return R.chi[s];
    else return (typename Row::value_type)0;
}
// r_y of the source in column s (0 in the lean pass's rows)
template <typename Row>
__device__ __forceinline__ typename Row::value_type ry_of(const Row& R, int s)
{
    if constexpr (Row::kRYS) return R.ry[s];
    else return (typename Row::value_type)0;
}

struct WaveInfo {  // per wavefront and staged row: ranges over its 64 sources
    int fxmin, fxmax, fymin, fymax, c1min, c1max;
    int ry0;       // 1 if every source has v_y integral (r_y = 0)
    int pad;
};

__device__ __forceinline__ WaveInfo merge(const WaveInfo& a, const WaveInfo& b)
{
    return WaveInfo{min(a.fxmin, b.fxmin), max(a.fxmax, b.fxmax), min(a.fymin, b.fymin),
                    max(a.fymax, b.fymax), min(a.c1min, b.c1min), max(a.c1max, b.c1max),
                    a.ry0 & b.ry0, 0};
}

// Accumulator type of the FIFO for storage type T.  FP32 storage keeps FP32
// accumulators: with the per-node primitives in FP64, FP64 accumulators did
// not lower the FP32 form's error against FP64 on the seeded planar tubes.
template <typename T>
using Acc = T;

template <typename T, int L, bool SP = false>
struct Fifo {
    static constexpr int NS = 2 * L + 1;
    T a[NS][kNV];        // slot o + L: destination row (current source row) + o
    YLaneSum<T> g[NS];   // y-lane momenta per slot
    T x[SP ? NS : 1];    // two gases: the species moment m chi per slot

    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int o = 0; o < NS; ++o) {
#pragma unroll
            for (int c = 0; c < kNV; ++c) a[o][c] = (T)0;
            g[o].zero();
            if constexpr (SP) x[o] = (T)0;
        }
    }
    // the oldest slot is written out: every slot moves down by one
    __device__ __forceinline__ void shift()
    {
#pragma unroll
        for (int o = 0; o + 1 < NS; ++o) {
#pragma unroll
            for (int c = 0; c < kNV; ++c) a[o][c] = a[o + 1][c];
            g[o] = g[o + 1];
            if constexpr (SP) x[o] = x[o + 1];
        }
#pragma unroll
        for (int c = 0; c < kNV; ++c) a[NS - 1][c] = (T)0;
        g[NS - 1].zero();
        if constexpr (SP) x[NS - 1] = (T)0;
    }
    // y-momentum of the oldest slot
    __device__ __forceinline__ T py0() const { return (T)(a[0][kPyv] + g[0].total()); }
};

// Add to the FIFO slot `slot` (differs between lanes) for slots in the
// wavefront-uniform range [lo, hi]: each slot in range takes a select, so the
// FIFO keeps compile-time indices (registers).  Slots out of range occur only
// with reach > H (reported).
template <typename A, typename T, int L, bool SP>
__device__ __forceinline__ void fifo_add_sel(Fifo<A, L, SP>& f, int slot, int lo, int hi, T r, T px, T pyv, T e,
                                             T xs = (T)0)
{
#pragma unroll
    for (int o = 0; o < 2 * L + 1; ++o) {
        if (o < lo || o > hi) continue;
        const bool h = slot == o;
        f.a[o][kR] += (A)(h ? r : (T)0);
        f.a[o][kPx] += (A)(h ? px : (T)0);
        f.a[o][kPyv] += (A)(h ? pyv : (T)0);
        f.a[o][kE] += (A)(h ? e : (T)0);
        if constexpr (SP) f.x[o] += (A)(h ? xs : (T)0);
    }
}

template <typename A, typename T, int L, bool SP>
__device__ __forceinline__ void fifo_add_g(Fifo<A, L, SP>& f, int slot, int lo, int hi, T v)
{
#pragma unroll
    for (int o = 0; o < 2 * L + 1; ++o) {
        if (o < lo || o > hi) continue;
        f.g[o].add((A)(slot == o ? v : (T)0));
    }
}

template <typename T>
__device__ __forceinline__ T fmaT(T a, T b, T c);
template <>
__device__ __forceinline__ float fmaT<float>(float a, float b, float c)
{
    return __builtin_fmaf(a, b, c);
}
template <>
__device__ __forceinline__ double fmaT<double>(double a, double b, double c)
{
    return __builtin_fma(a, b, c);
}

// The fast and the row paths add every packet class through the two helpers
// below, with fixed expressions (explicit fused multiply-adds, no automatic
// contraction).  A destination whose packets all come from sources of one
// floor(v_x) and c'_1 then gets the same bits whichever path its wavefront
// takes: the other classes add exact zeros.  Without this, wavefronts next to
// a transition would round an at-rest region differently from their
// neighbours, and the 1-ulp differences grow into momentum noise that flips
// floor(v_x) between -1 and 0.
//
// One +-c pair of x-lane packets: masses mp (+c) and mm (-c) into slot o.
// The pair's momentum m c' enters as (mp - mm) c, exactly zero for mirrored
// packets of equal mass.
template <typename A, typename T, int L, bool NOVY, bool SP>
__device__ __forceinline__ void add_xpair(Fifo<A, L, SP>& f, int o, T mp, T mm, T vxp, T vxm, T vyp, T vym, T cc,
                                          T zp, T zm, T xp = (T)0, T xm = (T)0)
{
#pragma clang fp contract(off)
    f.a[o][kR] += (A)(mp + mm);
    f.a[o][kPx] += (A)fmaT(mp - mm, cc, fmaT(mp, vxp, mm * vxm));
    if (!NOVY) f.a[o][kPyv] += (A)fmaT(mp, vyp, mm * vym);
    f.a[o][kE] += (A)fmaT(mp, zp, mm * zm);
    if constexpr (SP) f.x[o] += (A)fmaT(mp, xp, mm * xm);
}

// The +-c y-lane packets of NQ x-corner sources (masses m[q], kk = K + c^2/2)
// into slots op (+c) and om (-c); summed over the corners first, in order.
template <typename A, typename T, int L, int NQ, bool NOVY, bool SP>
__device__ __forceinline__ void add_ylanes(Fifo<A, L, SP>& f, int op, int om, const T (&m)[NQ], const T (&vx)[NQ],
                                           const T (&vy)[NQ], const T (&kk)[NQ], T cc, const T* xq = nullptr)
{
#pragma clang fp contract(off)
    T msum = m[0], pr = m[0] * vx[0], py = m[0] * vy[0];
#pragma unroll
    for (int q = 1; q < NQ; ++q) {
        msum += m[q];
        pr = fmaT(m[q], vx[q], pr);
        py = fmaT(m[q], vy[q], py);
    }
    T xsum = (T)0;
    if constexpr (SP) {
        xsum = m[0] * xq[0];
#pragma unroll
        for (int q = 1; q < NQ; ++q) xsum = fmaT(m[q], xq[q], xsum);
    }
    const T gm = msum * cc;
#pragma unroll
    for (int sg = -1; sg <= 1; sg += 2) {
        const int o = sg > 0 ? op : om;
        const T scc = sg > 0 ? cc : -cc;
        T pe;
        if (NOVY) {  // v_y = 0: K + c^2/2 + s c v_y is kk exactly
            pe = m[0] * kk[0];
#pragma unroll
            for (int q = 1; q < NQ; ++q) pe = fmaT(m[q], kk[q], pe);
        } else {
            pe = m[0] * fmaT(scc, vy[0], kk[0]);
#pragma unroll
            for (int q = 1; q < NQ; ++q) pe = fmaT(m[q], fmaT(scc, vy[q], kk[q]), pe);
        }
        f.a[o][kR] += (A)msum;
        f.a[o][kPx] += (A)pr;
        if (!NOVY) f.a[o][kPyv] += (A)py;
        f.g[o].add((A)(sg > 0 ? gm : -gm));
        f.a[o][kE] += (A)pe;
        if constexpr (SP) f.x[o] += (A)xsum;
    }
}

// The rest-group packets (square set with a rest level) of NQ x-corner
// sources (masses m[q], energy K[q]) into slot o; summed over the corners
// first, in order, like add_ylanes.
template <typename A, typename T, int L, int NQ, bool NOVY, bool SP>
__device__ __forceinline__ void add_rest(Fifo<A, L, SP>& f, int o, const T (&m)[NQ], const T (&vx)[NQ],
                                         const T (&vy)[NQ], const T (&K)[NQ], const T* xq = nullptr)
{
#pragma clang fp contract(off)
    T msum = m[0], pr = m[0] * vx[0], py = m[0] * vy[0], pe = m[0] * K[0];
#pragma unroll
    for (int q = 1; q < NQ; ++q) {
        msum += m[q];
        pr = fmaT(m[q], vx[q], pr);
        py = fmaT(m[q], vy[q], py);
        pe = fmaT(m[q], K[q], pe);
    }
    f.a[o][kR] += (A)msum;
    f.a[o][kPx] += (A)pr;
    if (!NOVY) f.a[o][kPyv] += (A)py;
    f.a[o][kE] += (A)pe;
    if constexpr (SP) {
        T xsum = m[0] * xq[0];
#pragma unroll
        for (int q = 1; q < NQ; ++q) xsum = fmaT(m[q], xq[q], xsum);
        f.x[o] += (A)xsum;
    }
}

// Rest-group mass at x corner kc of the source in column s: d_0 = rq (d_1 +
// d_2) of the staged level masses; and its energy per unit mass, K.
template <typename T, bool SP, bool RYS>
__device__ __forceinline__ T rest_mass(const MRow<T, SP, RYS>& R, int kc, int s, T rq)
{
    return rq * (R.m[0][kc][s] + R.m[1][kc][s]);
}
template <typename T, bool SP, bool RYS>
__device__ __forceinline__ T rest_k(const MRow<T, SP, RYS>& R, int s)
{
    const int c1 = mc1(R.pk[s]);
    return R.kk[0][s] - (T)0.5 * (T)(c1 * c1);
}

// Window where every source has floor(v_y) = FY, floor(v_x) in {fx - NKX + 2,
// fx} and c'_1 in {S0, S0 + NSP - 2}: the lanes of the window have speeds
// S0 .. S0 + NSP - 1, four per speed (+-x, +-y), and a source puts its level-1
// weight d_1 on speed c'_1 and d_2 on c'_1 + 1 (zero on the others); its x
// corners k_x = 0, 1 sit at x displacement floor(v_x) + k_x, i.e. at corners
// -1 .. 1 relative to fx.  Every packet class then has a compile-time column
// offset and FIFO slot.  NSP = 2, NKX = 2 is the uniform window.
// RY0: every source has r_y = 0, so the corners k_y = 1 carry no mass (eq. 29)
// and are skipped; with FY = 0 also v_y = 0 and the m v_y terms vanish.  The
// sums are the same, term for term.  REST: the rest group's packets (from the
// sources at x displacement floor(v_x) + k_x, into row FY + k_y) follow the
// lanes.  YM > 0: floor(v_y) is one of FY .. FY + YM per source (where v_y
// changes sign, YM = 1, or next to a region moving at |v_y| >= 1); the
// corners k_y = 0, 1 of a source then sit at rows FY + d with d =
// floor(v_y) - FY + k_y in 0 .. YM + 1, and each packet class is taken once
// per d with the source's weight for that row (zero for the rows it does not
// reach).  XCHK: only the sources with floor(v_x) = fx count (a window that
// mixes floor(v_x) takes one call per value).
template <typename T, int L, int FY, int S0, int NSP, int NKX, bool RY0, bool REST, int YM = 0,
          bool XCHK = false, bool SP, bool RYS>
__device__ __forceinline__ void gather_fast(const MRow<T, SP, RYS>& R, int lane, int fx, Fifo<Acc<T>, L, SP>& f,
                                            T rq)
{
#pragma clang fp contract(off)
    static_assert(!(YM && RY0), "a y-mixed window has sources with r_y != 0");
    static_assert(!XCHK || NKX == 2, "XCHK takes one value of floor(v_x) per call");
    constexpr bool UNI = NSP == 2;
    constexpr bool NOVY = RY0 && FY == 0;
    constexpr int NKY = YM ? YM + 2 : (RY0 ? 1 : 2);  // row offsets d of the packets (k_y, plus YM)
    constexpr int K0 = NKX == 3 ? -1 : 0;  // first x corner relative to floor(v_x) = fx
    const int base = lane - fx;  // staged column of x displacement fx + a is base - a
    // weight of row offset d for the source in column s with y fraction ry
    // (1 - r_y at its k_y = 0, r_y at k_y = 1)
    auto ywt = [&](int s, T ry, int d) -> T {
        if constexpr (YM > 0) {
            const int k = d - (mfy(R.pk[s]) - FY);
            return k == 0 ? (T)1 - ry : (k == 1 ? ry : (T)0);
        } else {
            return d ? ry : (T)1 - ry;
        }
    };
    // v_y of the source in column s
    auto vyof = [&](int s, T ry) -> T {
        if constexpr (YM > 0) return (T)mfy(R.pk[s]) + ry;
        else return (T)FY + ry;
    };
    // level (0: c'_1, 1: c'_2) that the source in column s has at speed
    // S0 + j, or -1 (no lane of that speed)
    auto level = [&](int s, int j) -> int {
        if (UNI) return j;
        const int l = S0 + j - mc1(R.pk[s]);
        return (l == 0 || l == 1) ? l : -1;
    };
    // packet mass of the source in column s at x corner k (relative to fx) and
    // speed S0 + j; with NKX = 3 a source may have floor(v_x) = fx - 1
    auto mass = [&](int s, int j, int k) -> T {
        const int l = level(s, j);
        // the source's own corner (XCHK: only sources with floor(v_x) = fx count)
        const int kc = XCHK ? (mfx(R.pk[s]) == fx ? k : -1) : (NKX == 2 ? k : k + fx - mfx(R.pk[s]));
        if (UNI && NKX == 2 && !XCHK) return R.m[l][kc][s];
        const T v = R.m[l < 0 ? 0 : l][kc < 0 ? 0 : (kc > 1 ? 1 : kc)][s];
        return (l >= 0 && kc >= 0 && kc <= 1) ? v : (T)0;
    };
    auto kkof = [&](int s, int j) -> T {
        const int l = level(s, j);
        return R.kk[l < 0 ? 0 : l][s];  // any finite value when the mass is zero
    };
#pragma unroll
    for (int j = 0; j < NSP; ++j) {
        const int c = S0 + j;
        const T cc = (T)c;
        // x-lanes: destination row FY + ky, source columns base - (kx +- c)
#pragma unroll
        for (int kx = K0; kx < 2; ++kx) {
            const int sp = base - (kx + c), sm = base - (kx - c);
            const T bp = mass(sp, j, kx), bm = mass(sm, j, kx);
            const T vxp = R.vx[sp], vxm = R.vx[sm];
            const T ryp = ry_of(R, sp), rym = ry_of(R, sm);
            const T vyp = vyof(sp, ryp), vym = vyof(sm, rym);
            const T zp = fmaT(cc, vxp, kkof(sp, j)), zm = fmaT(-cc, vxm, kkof(sm, j));
#pragma unroll
            for (int ky = 0; ky < NKY; ++ky) {
                const T mp = RY0 ? bp : bp * ywt(sp, ryp, ky);
                const T mm = RY0 ? bm : bm * ywt(sm, rym, ky);
                if constexpr (SP)
                    add_xpair<Acc<T>, T, L, NOVY>(f, FY + ky + L, mp, mm, vxp, vxm, vyp, vym, cc, zp, zm,
                                                  chi_of(R, sp), chi_of(R, sm));
                else
                    add_xpair<Acc<T>, T, L, NOVY>(f, FY + ky + L, mp, mm, vxp, vxm, vyp, vym, cc, zp, zm);
            }
        }
        // y-lanes: source columns base - kx
        T b[NKX], ry[NKX], vx[NKX], vy[NKX], kk[NKX], xq[NKX];
#pragma unroll
        for (int q = 0; q < NKX; ++q) {
            const int kx = K0 + q, sq = base - kx;
            b[q] = mass(sq, j, kx);
            ry[q] = ry_of(R, sq);
            vx[q] = R.vx[sq];
            vy[q] = vyof(sq, ry[q]);
            kk[q] = kkof(sq, j);
            xq[q] = chi_of(R, sq);
        }
#pragma unroll
        for (int ky = 0; ky < NKY; ++ky) {
            T m[NKX];
#pragma unroll
            for (int q = 0; q < NKX; ++q) m[q] = RY0 ? b[q] : b[q] * ywt(base - (K0 + q), ry[q], ky);
            add_ylanes<Acc<T>, T, L, NKX, NOVY>(f, FY + ky + c + L, FY + ky - c + L, m, vx, vy, kk, cc, xq);
        }
    }
    if constexpr (REST) {  // rest group: source columns base - kx, row FY + ky
        T b[NKX], ry[NKX], vx[NKX], vy[NKX], kr[NKX], xq[NKX];
#pragma unroll
        for (int q = 0; q < NKX; ++q) {
            const int kx = K0 + q, sq = base - kx;
            // the source's own corner (XCHK: only sources with floor(v_x) = fx count)
            const int kc = XCHK ? (mfx(R.pk[sq]) == fx ? kx : -1) : (NKX == 2 ? kx : kx + fx - mfx(R.pk[sq]));
            const T v = rest_mass(R, kc < 0 ? 0 : (kc > 1 ? 1 : kc), sq, rq);
            b[q] = (kc >= 0 && kc <= 1) ? v : (T)0;
            ry[q] = ry_of(R, sq);
            vx[q] = R.vx[sq];
            vy[q] = vyof(sq, ry[q]);
            kr[q] = rest_k(R, sq);
            xq[q] = chi_of(R, sq);
        }
#pragma unroll
        for (int ky = 0; ky < NKY; ++ky) {
            T m[NKX];
#pragma unroll
            for (int q = 0; q < NKX; ++q) m[q] = RY0 ? b[q] : b[q] * ywt(base - (K0 + q), ry[q], ky);
            add_rest<Acc<T>, T, L, NKX, NOVY>(f, FY + ky + L, m, vx, vy, kr, xq);
        }
    }
}

// Rows where every source seen by this wavefront has floor(v_y) = FY: the
// FIFO slot of every packet is known at compile time up to c'_1, which is
// taken from its (short) range [clo, chi] in unrolled branches; floor(v_x)
// and c'_1 may vary along the row.  Packets are taken per class (level, k_x,
// floor(v_x) = F, speed C): the x-lane pair +-C of a class comes from the two
// sources at x displacement k_x + F -+ C, and counts when that source has this
// F and speed C on this level (zero mass otherwise).  With chk (uniform), a
// source counts only if its floor(v_y) is FY as well: two such calls, for FY
// and FY + 1, take a window whose floor(v_y) has two adjacent values.  REST:
// the rest group's packets follow the lanes, in the fast path's order.
template <typename T, int L, int FY, bool REST, bool SP, bool RYS, bool RY0 = false>
__device__ __forceinline__ void gather_rows(const MRow<T, SP, RYS>& R, int lane, Fifo<Acc<T>, L, SP>& f, int fxlo,
                                            int fxhi, int clo, int chi, bool chk, T rq)
{
#pragma clang fp contract(off)
    // RY0 (FY = 0, every source with v_y = 0): the k_y = 1 corners carry no
    // mass and are skipped, and no packet carries m v_y; the other packets
    // are added in the same order, so the sums are bit for bit those of the
    // full form (which adds exact zeros for the skipped ones)
    constexpr bool NOVY = RY0 && FY == 0;
    constexpr int NKY = RY0 ? 1 : 2;
    const int nfx = fxhi - fxlo;
#pragma unroll
    for (int lev = 0; lev < 2; ++lev) {
        const int cl = clo + lev, ch = chi + lev;  // speeds of this level in the window
#pragma unroll
        for (int kx = 0; kx < 2; ++kx) {
            for (int i = 0; i <= nfx; ++i) {
                const int F = fxlo + i;
                for (int C = cl; C <= ch; ++C) {
                    const int sp = lane - (kx + F + C), sm = lane - (kx + F - C);
                    const int pkp = R.pk[sp], pkm = R.pk[sm];
                    const bool okp = mfx(pkp) == F && mc1(pkp) + lev == C && (!chk || mfy(pkp) == FY);
                    const bool okm = mfx(pkm) == F && mc1(pkm) + lev == C && (!chk || mfy(pkm) == FY);
                    const T bp = okp ? R.m[lev][kx][sp] : (T)0, bm = okm ? R.m[lev][kx][sm] : (T)0;
                    const T vxp = R.vx[sp], vxm = R.vx[sm];
                    const T ryp = ry_of(R, sp), rym = ry_of(R, sm);
                    const T vyp = (T)FY + ryp, vym = (T)FY + rym;
                    const T cc = (T)C;
                    const T zp = fmaT(cc, vxp, R.kk[lev][sp]), zm = fmaT(-cc, vxm, R.kk[lev][sm]);
#pragma unroll
                    for (int ky = 0; ky < NKY; ++ky) {
                        const T mp = bp * (ky ? ryp : (T)1 - ryp), mm = bm * (ky ? rym : (T)1 - rym);
                        if constexpr (SP)
                            add_xpair<Acc<T>, T, L, NOVY>(f, FY + ky + L, mp, mm, vxp, vxm, vyp, vym, cc, zp, zm,
                                                          chi_of(R, sp), chi_of(R, sm));
                        else
                            add_xpair<Acc<T>, T, L, NOVY>(f, FY + ky + L, mp, mm, vxp, vxm, vyp, vym, cc, zp, zm);
                    }
                }
            }
        }
        // y-lanes: the corners k_x = 0, 1 of floor(v_x) = F sit at x
        // displacement F and F + 1
        for (int i = 0; i <= nfx; ++i) {
            const int F = fxlo + i;
            const int s0 = lane - F, s1 = lane - F - 1;
            const int pk0 = R.pk[s0], pk1 = R.pk[s1];
            const bool ok0 = mfx(pk0) == F && (!chk || mfy(pk0) == FY);
            const bool ok1 = mfx(pk1) == F && (!chk || mfy(pk1) == FY);
            const int c0 = mc1(pk0) + lev, c1 = mc1(pk1) + lev;
            const T ry[2] = {ry_of(R, s0), ry_of(R, s1)};
            const T b0 = ok0 ? R.m[lev][0][s0] : (T)0, b1 = ok1 ? R.m[lev][1][s1] : (T)0;
            const T vx[2] = {R.vx[s0], R.vx[s1]};
            const T vy[2] = {(T)FY + ry[0], (T)FY + ry[1]};
            const T kk[2] = {R.kk[lev][s0], R.kk[lev][s1]};
            const T xq[2] = {chi_of(R, s0), chi_of(R, s1)};
#pragma unroll
            for (int C = 0; C <= 3 + 1; ++C) {  // speed of this level, static
                if (C < cl || C > ch) continue;
                if (FY + NKY - 1 + C > L || FY - C < -L) continue;  // out of the FIFO: redone / reported
                const T w0 = c0 == C ? b0 : (T)0, w1 = c1 == C ? b1 : (T)0;
                const T cc = (T)C;
#pragma unroll
                for (int ky = 0; ky < NKY; ++ky) {
                    const T m[2] = {w0 * (ky ? ry[0] : (T)1 - ry[0]), w1 * (ky ? ry[1] : (T)1 - ry[1])};
                    add_ylanes<Acc<T>, T, L, 2, NOVY>(f, FY + ky + C + L, FY + ky - C + L, m, vx, vy, kk, cc, xq);
                }
            }
        }
    }
    if constexpr (REST) {  // rest group: corners k_x = 0, 1 of floor(v_x) = F at F and F + 1
        for (int i = 0; i <= nfx; ++i) {
            const int F = fxlo + i;
            const int s0 = lane - F, s1 = lane - F - 1;
            const int pk0 = R.pk[s0], pk1 = R.pk[s1];
            const bool ok0 = mfx(pk0) == F && (!chk || mfy(pk0) == FY);
            const bool ok1 = mfx(pk1) == F && (!chk || mfy(pk1) == FY);
            const T ry[2] = {ry_of(R, s0), ry_of(R, s1)};
            const T b0 = ok0 ? rest_mass(R, 0, s0, rq) : (T)0, b1 = ok1 ? rest_mass(R, 1, s1, rq) : (T)0;
            const T vx[2] = {R.vx[s0], R.vx[s1]};
            const T vy[2] = {(T)FY + ry[0], (T)FY + ry[1]};
            const T kr[2] = {rest_k(R, s0), rest_k(R, s1)};
            const T xq[2] = {chi_of(R, s0), chi_of(R, s1)};
#pragma unroll
            for (int ky = 0; ky < NKY; ++ky) {
                const T m[2] = {b0 * (ky ? ry[0] : (T)1 - ry[0]), b1 * (ky ? ry[1] : (T)1 - ry[1])};
                add_rest<Acc<T>, T, L, 2, NOVY>(f, FY + ky + L, m, vx, vy, kr, xq);
            }
        }
    }
}

// Any mix of floor(v) and c'_1 around the destination (floor(v_y) varies
// across the wavefront, i.e. the flow is not planar here): examine the staged
// sources at x displacements [alo, ahi] (all that the window's packets can
// have, within the halo) and every packet that reaches this column.
// [fylo, fyhi] and [clo, chi] are the window's ranges of floor(v_y) and c'_1:
// each packet class then reaches one or two FIFO slots, and only those are
// visited.  REST: the set has a rest group, whose packets (mass
// rq (d_1 + d_2) per corner, energy K) move like the y-lanes with c' = 0.
template <typename T, int L, bool REST, bool SP>
__device__ void gather_general(const MRow<T, SP>& R, int lane, Fifo<Acc<T>, L, SP>& f, int alo, int ahi, int fylo,
                               int fyhi, int clo, int chi, T rq)
{
#pragma clang fp contract(off)
#pragma unroll 1
    for (int a = alo; a <= ahi; ++a) {  // x displacements the window's packets can have
        const int s = lane - a;
        const int pk = R.pk[s];
        const int fx = mfx(pk), fy = mfy(pk), c1 = mc1(pk), c2 = c1 + 1;
        const T vx = R.vx[s], ry = R.ry[s];
        const T vy = (T)fy + ry;
        const T xs = chi_of(R, s);  // two gases: mass fraction of gas 1
#pragma unroll 1
        for (int kx = 0; kx < 2; ++kx) {
            const int cx = a - fx - kx;  // x-lane speed needed to land here
            // x-lanes with c' = cx: +-c1 (both when c1 = 0) or +-c2
            const int n1 = (cx == c1 || cx == -c1) ? (c1 == 0 ? 2 : 1) : 0;
            const int n2 = (cx == c2 || cx == -c2) ? 1 : 0;
            if (n1 + n2 > 0) {
                const int l = n1 > 0 ? 0 : 1;
                const T w = (T)(n1 + n2) * R.m[l][kx][s];
                const T cc = (T)cx;
                const T zx = fmaT(cc, vx, R.kk[l][s]);
#pragma unroll 1
                for (int ky = 0; ky < 2; ++ky) {
                    const T m = w * (ky ? ry : (T)1 - ry);
                    fifo_add_sel<Acc<T>, T, L>(f, fy + ky + L, fylo + ky + L, fyhi + ky + L, m, m * (vx + cc),
                                               m * vy, m * zx, m * xs);
                }
            }
            if (cx == 0) {  // y-lanes (and the rest group) move in x by fx + kx only
                if constexpr (REST) {
                    const T mr = rq * (R.m[0][kx][s] + R.m[1][kx][s]);
                    const T zr = R.kk[0][s] - (T)0.5 * (T)(c1 * c1);  // K
#pragma unroll 1
                    for (int ky = 0; ky < 2; ++ky) {
                        const T m = mr * (ky ? ry : (T)1 - ry);
                        fifo_add_sel<Acc<T>, T, L>(f, fy + ky + L, fylo + ky + L, fyhi + ky + L, m, m * vx,
                                                   m * vy, m * zr, m * xs);
                    }
                }
#pragma unroll 1
                for (int l = 0; l < 2; ++l) {
                    const int c = l == 0 ? c1 : c2;
#pragma unroll 1
                    for (int sg = -1; sg <= 1; sg += 2) {
                        const T cc = (T)(sg * c);
                        const T zy = fmaT(cc, vy, R.kk[l][s]);
#pragma unroll 1
                        for (int ky = 0; ky < 2; ++ky) {
                            const T m = R.m[l][kx][s] * (ky ? ry : (T)1 - ry);
                            const int slot = fy + ky + sg * c + L;
                            // the window's range of this packet class's slot (uniform)
                            const int lo = fylo + ky + (sg > 0 ? clo + l : -(chi + l)) + L;
                            const int hi = fyhi + ky + (sg > 0 ? chi + l : -(clo + l)) + L;
                            fifo_add_sel<Acc<T>, T, L>(f, slot, lo, hi, m, m * vx, m * vy, m * zy, m * xs);
                            fifo_add_g<Acc<T>, T, L>(f, slot, lo, hi, m * cc);
                        }
                    }
                }
            }
        }
    }
}

template <typename T, int NF>
__device__ __forceinline__ void load_node(const T* __restrict__ Y, int64_t nn, int64_t q, T (&m)[NF])
{
    m[0] = Y[q];
    m[1] = Y[nn + q];
    m[2] = Y[2 * nn + q];
    m[3] = Y[3 * nn + q];
    if constexpr (NF > 4) m[4] = Y[4 * nn + q];
}

// Per-tile flag bits of the square-lattice passes.  The short pass writes
// kFlagFar and kFlagReach of every tile it claims (a tile it leaves to the
// full pass gets both: its sources are not looked at); the full pass reads
// them and rewrites only kFlagKeep, the tile still needs the full FIFO, which
// the next step's short pass reads.  In the lean pass's flag words the short
// pass keeps kFlagKeep for the tiles it computed whose sources the lean pass
// cannot take (march_tile's kFlagNotLean), and the next step's lean pass
// leaves those to it at once.
constexpr int kFlagFar = 1, kFlagReach = 2, kFlagKeep = 4, kFlagNotLean = 8;
// flags_lean: the tile is in this step's list for the full pass (row chunks)
constexpr int kFlagFullListed = 16;

// Work of one window of a wavefront on the paths of march_tile, in units of
// about half a uniform window (the fast instances' packet classes: speeds x
// x corners x row offsets), summed over a tile's staged rows per wavefront;
// a tile's work is its busiest wavefront's (the row barriers wait for it).
constexpr int kUnitFast = 2, kUnitFastMix = 3, kUnitXSplit = 5, kUnitYMix = 3, kUnitYXSplit = 9,
              kUnitWide = 14, kUnitRows = 9, kUnitGeneral = 32;

// Row chunks of heavy tiles (plain form of the short and full passes).  A
// tile whose windows take the slow paths costs the pass up to several times
// the mean tile, and a pass lasts as long as its slowest block: such a tile
// is cut into up to kSplitMax chunks of rows, which other blocks claim, each
// marching its own rows plus the L halo rows on each side.  The short pass
// cuts a tile by the work the last pass that computed it measured there (one
// chunk more per kSplitWork units for the rows of a whole tile: about three
// times a uniform tile's, so that only tiles that would outlast the pass's
// mean load per block are cut, each chunk adding 2 L halo rows); the full
// pass, which takes few tiles, cuts each of its tiles into as many chunks as
// leave every resident block about one.  A chunk's per-tile results (field
// sums, reach, error and flag bits) go to a slot of their own; the tile's
// last chunk to finish adds the slots in chunk order into the tile's row of
// partials, so the totals do not depend on which block ran which chunk.
// Every node of a chunk is summed exactly as in the whole tile (the FIFO adds
// a destination row's packets in source-row order whatever row the march
// starts from).
constexpr int kSplitWork = 150;
constexpr int kWorkListed = 1 << 30;  // work word: the tile is in this step's list

// Whether the next pass must compute the tile of destination rows
// [Y0, ylast) whose row chunk ty0 = Y0 / sy starts at flag index tbase +
// ty0 * tiles_x + tx (row chunks of sy rows, column strips tiles_x wide),
// after a pass that staged LP rows on each side of its tiles and wrote
// `flags`.  A source up to H rows away can reach the tile: the rows
// [Y0 - H, Y0 - LP) and [ylast + LP, ylast + H), mapped by the y boundary,
// belong to other row chunks (or the same one).  A source there that reaches
// the tile has a y-reach beyond LP, so the chunk owning its row raised
// kFlagReach: a periodic or clamped halo row is the very source it stands
// for, and a mirror image beyond a wall reaches inside only with packets
// whose mirror images, from the node inside, reach as far out (zero-mass
// corners aside, which add nothing).  The tile is computed again if its own
// pass was incomplete or any such chunk raised kFlagReach.
template <int LP>
__device__ __forceinline__ bool needs_pass(const int* __restrict__ flags, int64_t tbase, int64_t tiles_x,
                                           int64_t tx, int64_t Y0, int64_t ylast, int sy, int64_t ny, int bc_y)
{
    if (flags[tbase + (Y0 / sy) * tiles_x + tx] & kFlagFar) return true;
#pragma unroll
    for (int i = 0; i < 2 * (kMH - LP); ++i) {
        const int d = i % (kMH - LP);
        const int64_t row = i < kMH - LP ? Y0 - kMH + d : ylast + LP + d;
        bool mir = false;
        const int64_t src = source_idx(row, ny, bc_y, &mir);
        if (flags[tbase + (src / sy) * tiles_x + tx] & kFlagReach) return true;
    }
    return false;
}

// One tile: destination columns [X0, X0 + 256 - 2H) and rows [Y0, Y0 + sy)
// (clipped to the grid) of grid g, marched from row Y0 - L to Y0 + sy + L - 1.
// Writes Yn and one row of per-tile partials (field sums, reach, error bits).
// Returns kFlag* bits (the same in every thread).  kFlagFar: the short pass
// cannot take some window of the tile: a y-displacement beyond the short FIFO
// (kLSmall), or a non-planar window (floor(v_y) not uniform, and the mixes
// the row path does not take), which only the full pass's paths handle.  With
// L = kLSmall the tile's output is then incomplete and must be recomputed
// with L = kLFull, which sums in the same order (bit-identical); with
// L = kLFull it tells that the tile still needs the full pass.  kFlagReach: a
// source in the first or last H of the tile's own destination rows has a
// y-reach beyond kLSmall, so it may reach destination rows of the
// neighbouring row chunks that their short passes complete without staging
// it (see needs_pass).  kFlagNotLean:
// some staged source has v_y != 0, c'_1 > 1 or a bad state (the lean pass
// would give the tile up).
// Contains block-wide barriers: every thread of the block must call it.
template <typename T, int L, bool WALLS, bool REST, bool SP>
__device__ __forceinline__ int march_tile(const T* __restrict__ Y, T* __restrict__ Yn, const Grid& g, const Consts& k,
                          int64_t X0, int64_t Y0, int sy, double* __restrict__ prow, int* cost = nullptr)
{
    // source rows staged per barrier: two (fewer barriers, two independent
    // per-source computations in flight)
    constexpr int RB = 2;
    constexpr int NF = SP ? 5 : 4;  // moment fields (two gases: rho chi after rho E)
    __shared__ MRow<T, SP> s_row[2][RB];
    __shared__ WaveInfo s_w[2][RB][kMNW];
    const int tid = threadIdx.x, lane64 = tid & 63, wid = tid >> 6;
    const T rq = REST ? (T)k.rest_q : (T)0;  // rest-group mass per unit of staged level mass
    const int64_t nx = g.nx, ny = g.ny, nn = nx * ny;
    const int64_t gx = X0 - kMH + tid;                           // this thread's source column
    bool mir_x = false;
    int64_t sx;
    if constexpr (WALLS) sx = source_idx(gx, nx, g.bc_x, &mir_x);
    else sx = g.bc_x == kBcPeriodic ? wrap_near(gx, nx) : clamp_idx(gx, nx);
    const bool dest = tid >= kMH && tid < kMTPB - kMH && gx < nx;
    const int64_t ylast = min(Y0 + (int64_t)sy, ny);  // destination rows [Y0, ylast)
    const int nrows = Y0 < ny ? (int)(ylast - Y0) + 2 * L : 0;
    constexpr int NS = 2 * L + 1;

    using A = Acc<T>;
    Fifo<A, L, SP> f;
    f.zero();
    double tot[NF] = {};
    int reach = 0, bad = 0, yfar = 0, yreach = 0, unlean = 0;
    int units = 0;  // work of this thread's wavefront's windows (see kUnit*)

    // moments of this thread's source column in row gy (halo rows and
    // columns mapped by the boundaries); *mir_y tells whether the row is a
    // mirror image beyond a wall.  Mirror images negate normal momentum when
    // the row is staged, so that the loads issued a row ahead are not waited for.
    auto load_src = [&](int64_t gy, T (&m)[NF], bool* mir_y) {
        int64_t yy;
        if constexpr (WALLS) yy = source_idx(gy, ny, g.bc_y, mir_y);
        else yy = g.bc_y == kBcPeriodic ? wrap_near(gy, ny) : clamp_idx(gy, ny);
        load_node<T, NF>(Y, nn, yy * nx + sx, m);
    };
    T cur[RB][NF], nxt[RB][NF];
    bool cur_my[RB] = {}, nxt_my[RB] = {};
#pragma unroll
    for (int u = 0; u < RB; ++u)
        if (u < nrows) load_src(Y0 - L + u, cur[u], &cur_my[u]);

    for (int r0 = 0; r0 < nrows; r0 += RB) {
        const int b = (r0 / RB) & 1;
#pragma unroll
        for (int u = 0; u < RB; ++u)
            if (r0 + RB + u < nrows) load_src(Y0 - L + r0 + RB + u, nxt[u], &nxt_my[u]);
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            if (r0 + u >= nrows) break;
            // stage this source row
            T mx = cur[u][1], my = cur[u][2];
            if constexpr (WALLS) {
                mx = mir_x ? -mx : mx;
                my = cur_my[u] ? -my : my;
            }
            const Src2<T> s = make_src2<T, REST, SP>(cur[u][0], mx, my, cur[u][3], k, cur[u][NF - 1]);
            const int pk = mpack(s.fx, s.fy, s.c1);
            s_row[b][u].vx[tid] = s.vx;
            s_row[b][u].ry[tid] = s.ry;
            s_row[b][u].m[0][0][tid] = s.m[0][0];
            s_row[b][u].m[0][1][tid] = s.m[0][1];
            s_row[b][u].m[1][0][tid] = s.m[1][0];
            s_row[b][u].m[1][1][tid] = s.m[1][1];
            s_row[b][u].kk[0][tid] = s.kk[0];
            s_row[b][u].kk[1][tid] = s.kk[1];
            s_row[b][u].pk[tid] = pk;
            if constexpr (SP) s_row[b][u].chi[tid] = s.chi;
            const int yr = axis_reach(s.fy, s.c1);
            reach = max(reach, max(axis_reach(s.fx, s.c1), yr));
            yfar |= yr > kLSmall ? 1 : 0;
            // a source in the first or last H of the tile's own destination
            // rows that reaches past the short FIFO: the neighbouring tiles'
            // short passes, which do not stage this row, may miss its packets
            // (every source row another tile's pass does not stage lies within
            // H rows of an edge of its own tile, after the boundary map)
            yreach |= (yr > kLSmall && r0 + u >= L && r0 + u < nrows - L &&
                       (r0 + u < L + kMH || r0 + u >= nrows - L - kMH)) ? 1 : 0;
            bad |= s.bad ? 1 : 0;
            unlean |= (s.bad || s.fy != 0 || s.ry != (T)0 || s.c1 > 1) ? 1 : 0;
            {
                const int ry0 = __all(s.ry == (T)0) ? 1 : 0;
                const int pk0 = __builtin_amdgcn_readfirstlane(pk);
                WaveInfo wi;
                if (__all(pk == pk0)) {  // the common case: one ballot instead of six reductions
                    wi = WaveInfo{mfx(pk0), mfx(pk0), mfy(pk0), mfy(pk0), mc1(pk0), mc1(pk0), ry0, 0};
                } else {
                    wi = WaveInfo{wave_min(s.fx), wave_max(s.fx), wave_min(s.fy), wave_max(s.fy),
                                  wave_min(s.c1), wave_max(s.c1), ry0, 0};
                }
                if (lane64 == 0) s_w[b][u][wid] = wi;
            }

        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            const int r = r0 + u;
            if (r >= nrows) break;
            // gather this row's packets into the FIFO
            WaveInfo w = s_w[b][u][wid];
            if (wid > 0) w = merge(w, s_w[b][u][wid - 1]);
            if (wid + 1 < kMNW) w = merge(w, s_w[b][u][wid + 1]);
            // the fast and row paths need every packet of the window inside the
            // FIFO (y) and the staged row (x); the full pass's general path
            // takes any window whose sources each reach <= H.
            const int c2max = w.c1max + 1;
            const bool fits_y = w.fymin - c2max >= -L && w.fymax + 1 + c2max <= L;
            const bool fits_small = w.fymin - c2max >= -kLSmall && w.fymax + 1 + c2max <= kLSmall;
            const bool fits_x = w.fxmin - c2max >= -kMH && w.fxmax + 1 + c2max <= kMH;
            const bool planar = fits_x && w.fymin == w.fymax && (w.fymin == 0 || w.fymin == -1) &&
                                w.c1max <= 3 && w.fxmax - w.fxmin <= 2;
            const bool rows_ok = planar && fits_y;
            // floor(v_y) in {-1, 0} (where v_y changes sign): the row path
            // once per value (other pairs of values take the full pass's
            // general path: their instances made the compiler spill the FIFO
            // on every path)
            const bool ymix_ok = fits_x && fits_y && w.fymin == -1 && w.fymax == 0 && w.c1max <= 3 &&
                                 w.fxmax - w.fxmin <= 2;
            // full pass: floor(v_y) taking two or three values in [-2, 1] (a
            // region moving at |v_y| >= 1 next to one at rest): the row path
            // once per value, as for {-1, 0}
            constexpr bool kWide = L == kLFull && sizeof(T) == 8;
            const bool ymulti_ok = L == kLFull && fits_x && fits_y && w.fymin >= -2 && w.fymax <= 1 &&
                                   w.fymax - w.fymin <= 2 && w.c1max <= 3 && w.fxmax - w.fxmin <= 2;
            // the short pass takes these windows and the planar ones within
            // its FIFO; a tile with any other window is flagged for the full pass
            if (!((planar || ymix_ok) && fits_small)) yfar = 1;
            if (dest && (fits_y || L == kLFull)) {
                // two adjacent values of c'_1 or of floor(v_x) keep compile-time
                // offsets; a window mixing both (rare in planar flows) takes the
                // row path, whose extra registers would otherwise cost occupancy
                const bool cmix = w.c1max == w.c1min + 1, xmix = w.fxmax == w.fxmin + 1;
                const bool mixes = (w.c1max == w.c1min || cmix) && (w.fxmax == w.fxmin || xmix) &&
                                   !(cmix && xmix) && (!cmix || w.c1min <= 2) && (!xmix || w.c1min <= 1);
                const bool fastw = rows_ok && mixes;
                // planar, c'_1 in {0, 1} or {1, 2} and floor(v_x) in {fx - 1, fx}:
                // the c'_1-mixed instance once per value of floor(v_x)
                const bool xsplitw = rows_ok && cmix && xmix && w.c1min <= 1;
                // floor(v_y) in {-1, 0} with the same mixes: the y-mixed
                // instances (three row offsets per packet class)
                const bool ymixw = ymix_ok && mixes && !xmix && w.c1max <= 1;
                // floor(v_y) in {-1, 0} and floor(v_x) in {fx - 1, fx} as well
                // (c'_1 <= 1): the y-mixed instance once per value of floor(v_x)
                const bool yxsplitw = ymix_ok && xmix && w.c1max <= 1;
                const bool widew = kWide && fits_x && fits_y && w.c1max <= 1 && w.fxmax - w.fxmin <= 1 &&
                                   w.fymax == 1 && (w.fymin == 0 || w.fymin == -1);
                units += yxsplitw ? kUnitYXSplit
                       : xsplitw ? kUnitXSplit
                       : fastw ? (cmix ? kUnitFastMix : kUnitFast)
                       : ymixw ? kUnitYMix
                       : widew ? kUnitWide
                       : (rows_ok || ymix_ok || ymulti_ok) ? kUnitRows * (w.fymax - w.fymin + 1)
                       : (L == kLFull ? kUnitGeneral : 0);
                if (yxsplitw) {
                    const auto& R = s_row[b][u];
                    if (w.c1min == w.c1max) {
                        if (w.c1min == 0) {
                            gather_fast<T, L, -1, 0, 2, 2, false, REST, 1, true>(R, tid, w.fxmin, f, rq);
                            gather_fast<T, L, -1, 0, 2, 2, false, REST, 1, true>(R, tid, w.fxmax, f, rq);
                        } else {
                            gather_fast<T, L, -1, 1, 2, 2, false, REST, 1, true>(R, tid, w.fxmin, f, rq);
                            gather_fast<T, L, -1, 1, 2, 2, false, REST, 1, true>(R, tid, w.fxmax, f, rq);
                        }
                    } else {
                        gather_fast<T, L, -1, 0, 3, 2, false, REST, 1, true>(R, tid, w.fxmin, f, rq);
                        gather_fast<T, L, -1, 0, 3, 2, false, REST, 1, true>(R, tid, w.fxmax, f, rq);
                    }
                } else if (xsplitw) {
                    const auto& R = s_row[b][u];
                    const int sel = (w.fymin == 0 ? (w.ry0 ? 0 : 1) : 2) * 2 + w.c1min;
                    switch (sel) {
    #define LB_XSPLIT(S, FYV, S0, RY)                                                                      \
        case S:                                                                                            \
            if constexpr ((FYV) - (S0) - 2 >= -L && (FYV) + 1 + (S0) + 2 <= L) {                            \
                gather_fast<T, L, FYV, S0, 3, 2, RY, REST, 0, true>(R, tid, w.fxmin, f, rq);          \
                gather_fast<T, L, FYV, S0, 3, 2, RY, REST, 0, true>(R, tid, w.fxmax, f, rq);          \
            }                                                                                              \
            break;
                        LB_XSPLIT(0, 0, 0, true) LB_XSPLIT(1, 0, 1, true)
                        LB_XSPLIT(2, 0, 0, false) LB_XSPLIT(3, 0, 1, false)
                        LB_XSPLIT(4, -1, 0, false) LB_XSPLIT(5, -1, 1, false)
    #undef LB_XSPLIT
                        default: break;  // not reached
                    }
                } else if (fastw || ymixw) {
                    const auto& R = s_row[b][u];
                    const int fx0 = w.fxmax;
                    const int sel = ((ymixw ? 3 : (w.fymin == 0 ? (w.ry0 ? 0 : 1) : 2)) * 2 + (xmix ? 1 : 0)) * 8 +
                                    (cmix ? 4 : 0) + w.c1min;
                    switch (sel) {
    #define LB_FAST(S, FYV, S0, NSP, NKX, RY, YM)                                                           \
        case S:                                                                                             \
            if constexpr ((FYV) - (S0) - (NSP) + 1 >= -L && (FYV) + (YM) + 1 + (S0) + (NSP) - 1 <= L)       \
                gather_fast<T, L, FYV, S0, NSP, NKX, RY, REST, YM>(R, tid, fx0, f, rq);                     \
            break;
    #define LB_FAST_SET(B, FYV, RY, YM)                                                                      \
        LB_FAST(B + 0, FYV, 0, 2, 2, RY, YM) LB_FAST(B + 1, FYV, 1, 2, 2, RY, YM)                            \
        LB_FAST(B + 2, FYV, 2, 2, 2, RY, YM) LB_FAST(B + 3, FYV, 3, 2, 2, RY, YM)                            \
        LB_FAST(B + 4, FYV, 0, 3, 2, RY, YM) LB_FAST(B + 5, FYV, 1, 3, 2, RY, YM)                            \
        LB_FAST(B + 6, FYV, 2, 3, 2, RY, YM)                                                                 \
        LB_FAST(B + 8, FYV, 0, 2, 3, RY, YM) LB_FAST(B + 9, FYV, 1, 2, 3, RY, YM)
                        LB_FAST_SET(0, 0, true, 0)
                        LB_FAST_SET(16, 0, false, 0)
                        LB_FAST_SET(32, -1, false, 0)
                        // y-mixed: uniform c'_1 0 or 1 and c'_1 in {0, 1} (the other
                        // instances made the compiler spill the short pass's FIFO)
                        LB_FAST(48 + 0, -1, 0, 2, 2, false, 1) LB_FAST(48 + 1, -1, 1, 2, 2, false, 1)
                        LB_FAST(48 + 4, -1, 0, 3, 2, false, 1)
    #undef LB_FAST_SET
    #undef LB_FAST
                        default: break;  // not reached: fastw and ymixw admit only the cases above
                    }
                } else if (widew) {
                    // full pass: floor(v_y) in {0, 1} or {-1, 0, 1} (next to a
                    // region moving at v_y >= 1), c'_1 <= 1: the y-mixed
                    // instances (YM = 1 from 0, YM = 2 from -1; speeds 0 .. 2,
                    // which also take a uniform c'_1), once per value of
                    // floor(v_x).  FP64 only: in FP32 their registers would
                    // cost the pass its second wavefront per SIMD.
                    if constexpr (kWide) {
                        const auto& R = s_row[b][u];
                        for (int fxq = w.fxmin; fxq <= w.fxmax; ++fxq) {
                            if (w.fymin == 0) {
                                gather_fast<T, L, 0, 0, 3, 2, false, REST, 1, true>(R, tid, fxq, f, rq);
                            } else {
                                gather_fast<T, L, -1, 0, 3, 2, false, REST, 2, true>(R, tid, fxq, f, rq);
                            }
                        }
                    }
                } else if (rows_ok || ymix_ok || ymulti_ok) {
                    // one call per value of floor(v_y) in the window (one
                    // call site per instance keeps the kernel's code compact)
                    const auto& R = s_row[b][u];
                    const bool chk = w.fymin != w.fymax;
                    if constexpr (L == kLFull) {
                        if (w.fymin <= -2)
                            gather_rows<T, L, -2, REST>(R, tid, f, w.fxmin, w.fxmax, w.c1min, w.c1max, chk, rq);
                    }
                    if (w.fymin <= -1 && w.fymax >= -1)
                        gather_rows<T, L, -1, REST>(R, tid, f, w.fxmin, w.fxmax, w.c1min, w.c1max, chk, rq);
                    if (w.fymin <= 0 && w.fymax >= 0)
                        gather_rows<T, L, 0, REST>(R, tid, f, w.fxmin, w.fxmax, w.c1min, w.c1max, chk, rq);
                    if constexpr (L == kLFull) {
                        if (w.fymax >= 1)
                            gather_rows<T, L, 1, REST>(R, tid, f, w.fxmin, w.fxmax, w.c1min, w.c1max, chk, rq);
                    }
                } else if (L == kLFull) {  // other windows: the short pass flags the tile (above)
                    gather_general<T, L, REST>(s_row[b][u], tid, f, max(-kMH, w.fxmin - c2max),
                                               min(kMH, w.fxmax + 1 + c2max), w.fymin, w.fymax, w.c1min, w.c1max,
                                               rq);
                }
            }
            // destination row (source row) - L is complete
            if (r >= 2 * L && dest) {
                const int64_t ty = Y0 + r - 2 * L;
                const int64_t q = ty * nx + gx;
                const T py = f.py0();
                Yn[q] = (T)f.a[0][kR];
                Yn[nn + q] = (T)f.a[0][kPx];
                Yn[2 * nn + q] = py;
                Yn[3 * nn + q] = (T)f.a[0][kE];
                tot[0] += (double)f.a[0][kR];
                tot[1] += (double)f.a[0][kPx];
                tot[2] += (double)py;
                tot[3] += (double)f.a[0][kE];
                if constexpr (SP) {
                    Yn[4 * nn + q] = (T)f.x[0];
                    tot[NF - 1] += (double)f.x[0];
                }
            }
            f.shift();
        }
#pragma unroll
        for (int u = 0; u < RB; ++u) {
#pragma unroll
            for (int c = 0; c < NF; ++c) cur[u][c] = nxt[u][c];
            if constexpr (WALLS) cur_my[u] = nxt_my[u];
        }
    }
    // per-tile partials: field sums (a fifth, rho chi, at index 6), reach, error bits
    __shared__ double s_sum[kMNW][NF];
    __shared__ int s_ir[kMNW][3];
#pragma unroll
    for (int c = 0; c < NF; ++c) tot[c] = wave_sum(tot[c]);
    reach = wave_max(reach);
    bad = wave_max(bad);
    units = wave_max(units);
    if (lane64 == 0) {
#pragma unroll
        for (int c = 0; c < NF; ++c) s_sum[wid][c] = tot[c];
        s_ir[wid][0] = reach;
        s_ir[wid][1] = bad;
        s_ir[wid][2] = units;
    }
    // (__syncthreads_or returns whether any value is non-zero, not their OR)
    const int far = (__syncthreads_or(yfar) ? kFlagFar : 0) | (__syncthreads_or(yreach) ? kFlagReach : 0) |
                    (__syncthreads_or(unlean) ? kFlagNotLean : 0);
    if (tid == 0) {
        int rr = 0, bb = 0;
        for (int c = 0; c < NF; ++c) {
            double t = s_sum[0][c];
            for (int w = 1; w < kMNW; ++w) t += s_sum[w][c];
            prow[c < 4 ? c : 6] = t;
        }
        int uu = 0;
        for (int w = 0; w < kMNW; ++w) {
            rr = max(rr, s_ir[w][0]);
            bb |= s_ir[w][1];
            uu = max(uu, s_ir[w][2]);
        }
        prow[4] = (double)rr;
        prow[5] = (double)((rr > kMH ? kErrReach : 0) | (bb ? kErrState : 0));
        if (cost) *cost = uu;
    }
    return far;
}

// The lean first pass: one tile, as march_tile, for x-planar flows.  It takes
// a tile only if every source it stages has v_y = 0 exactly (floor(v_y) = 0,
// r_y = 0) and c'_1 <= 1, and every window is one of the fast path's uniform
// or one-step-mixed cases: then a packet moves at most c'_2 <= 2 rows (the
// k_y = 1 corners carry no mass and are skipped, eq. 29 with r_y = 0), a FIFO
// of 2 kLLean + 1 = 5 slots holds every pending destination row, no packet
// carries m v_y, and r_y need not be staged.  Those savings, and one staged
// row per barrier, keep the registers and LDS of four wavefronts per SIMD.
// The packets go through the same gather_fast instances in the same source
// row order as in march_tile, so a tile it completes is bit-identical to the
// short pass's result.  At the first row that breaks these conditions the
// whole block gives the tile up (the decision rides on the row's barrier) and
// returns kFlagFar | kFlagReach: the short pass then computes it, and the
// tiles around it (see needs_pass).  Returns 0 when the tile is complete.
// Contains block-wide barriers: every thread of the block must call it.
constexpr int kLLean = 2;

// The element at byte offset `off` from p (p wave-uniform, off per lane):
// the form the hardware's scalar-base global loads and stores take.
template <typename T>
__device__ __forceinline__ T& at_byte(T* p, uint32_t off)
{
    return *(T*)((char*)p + off);
}
template <typename T>
__device__ __forceinline__ const T& at_byte(const T* p, uint32_t off)
{
    return *(const T*)((const char*)p + off);
}

// A wavefront's summary of one staged row in the lean pass, one int: its
// ranges of floor(v_x) (biased by 128, as mpack clamps them) and c'_1 (at
// most 15 is kept: the pass gives up any tile with c'_1 > 1), and kLeanStop.
constexpr int kLeanStop = 1 << 24;
__device__ __forceinline__ int lean_word(int fxmin, int fxmax, int c1min, int c1max, int stop)
{
    return (fxmin + 128) | ((fxmax + 128) << 8) | (min(c1min, 15) << 16) | (min(c1max, 15) << 20) | stop;
}
__device__ __forceinline__ int lean_fxmin(int w) { return (w & 255) - 128; }
__device__ __forceinline__ int lean_fxmax(int w) { return ((w >> 8) & 255) - 128; }
__device__ __forceinline__ int lean_c1min(int w) { return (w >> 16) & 15; }
__device__ __forceinline__ int lean_c1max(int w) { return (w >> 20) & 15; }

template <typename T, bool WALLS, bool REST, bool SP>
__device__ __forceinline__ int march_tile_lean(const T* __restrict__ Y, T* __restrict__ Yn, const Grid& g,
                                               const Consts& k, int64_t X0, int64_t Y0, int sy,
                                               double* __restrict__ prow)
{
    constexpr int L = kLLean;
    constexpr int NF = SP ? 5 : 4;
    __shared__ MRow<T, SP, false> s_row[2];
    // per wavefront and staged row: its ranges of floor(v_x) and c'_1, and
    // whether the tile must be given up (lean_word)
    __shared__ int4 s_wave[2];
    const int tid = threadIdx.x, lane64 = tid & 63, wid = tid >> 6;
    const T rq = REST ? (T)k.rest_q : (T)0;
    const int64_t nx = g.nx, ny = g.ny, nn = nx * ny;
    const int64_t gx = X0 - kMH + tid;
    bool mir_x = false;
    int64_t sx;
    if constexpr (WALLS) sx = source_idx(gx, nx, g.bc_x, &mir_x);
    else sx = g.bc_x == kBcPeriodic ? wrap_near(gx, nx) : clamp_idx(gx, nx);
    // byte offsets of the columns within a row: 32 bits (a square-lattice
    // grid is at most 2^28 nodes wide), added to a wave-uniform row address
    const uint32_t sxb = (uint32_t)sx * (uint32_t)sizeof(T), gxb = (uint32_t)gx * (uint32_t)sizeof(T);
    const bool dest = tid >= kMH && tid < kMTPB - kMH && gx < nx;
    const int64_t ylast = min(Y0 + (int64_t)sy, ny);
    const int nrows = Y0 < ny ? (int)(ylast - Y0) + 2 * L : 0;
    constexpr int NS = 2 * L + 1;

    using A = Acc<T>;
    Fifo<A, L, SP> f;
    f.zero();
    double tot[NF] = {};
    int reach = 0, far = 0;

    auto load_src = [&](int64_t gy, T (&m)[NF], bool* mir_y) {
        int64_t yy;
        if constexpr (WALLS) yy = source_idx(gy, ny, g.bc_y, mir_y);
        else yy = g.bc_y == kBcPeriodic ? wrap_near(gy, ny) : clamp_idx(gy, ny);
#pragma unroll
        for (int c = 0; c < NF; ++c) m[c] = at_byte(Y + (int64_t)c * nn + yy * nx, sxb);  // uniform row + column
    };
    // one source row in registers: row r + 1 is loaded into them as soon as
    // row r's primitives have read them, and arrives while row r is staged
    // and gathered (no copy of registers with loads in flight, which would
    // wait for them)
    T cur[NF];
    bool cur_my = false;
    if (nrows > 0) load_src(Y0 - L, cur, &cur_my);

    for (int r = 0; r < nrows; ++r) {
        const int b = r & 1;
        T mx = cur[1], my = cur[2];
        if constexpr (WALLS) {
            mx = mir_x ? -mx : mx;
            my = cur_my ? -my : my;
        }
        const Src2<T> s = make_src2<T, REST, SP, true>(cur[0], mx, my, cur[3], k, cur[NF - 1]);
        if (r + 1 < nrows) load_src(Y0 - L + r + 1, cur, &cur_my);
        const int pk = mpack(s.fx, s.fy, s.c1);
        MRow<T, SP, false>& R = s_row[b];
        R.vx[tid] = s.vx;
        R.m[0][0][tid] = s.m[0][0];
        R.m[0][1][tid] = s.m[0][1];
        R.m[1][0][tid] = s.m[1][0];
        R.m[1][1][tid] = s.m[1][1];
        R.kk[0][tid] = s.kk[0];
        R.kk[1][tid] = s.kk[1];
        R.pk[tid] = pk;
        if constexpr (SP) R.chi[tid] = s.chi;
        reach = max(reach, max(axis_reach(s.fx, s.c1), axis_reach(s.fy, s.c1)));  // as march_tile reports it
        // v_y = 0 exactly and c'_1 <= 1 (and a good state: bad ones are the short pass's to report)
        const bool ok = !s.bad && s.fy == 0 && s.ry == (T)0 && s.c1 <= 1;
        {
            const int pk0 = __builtin_amdgcn_readfirstlane(pk);
            int word;
            if (__all(pk == pk0))
                word = lean_word(mfx(pk0), mfx(pk0), mc1(pk0), mc1(pk0), 0);
            else
                word = lean_word(wave_min(s.fx), wave_max(s.fx), wave_min(s.c1), wave_max(s.c1), 0);
            // this row's sources, or the previous row's window (far), rule the tile out
            if (__any(!ok) || far) word |= kLeanStop;
            if (lane64 == 0) (&s_wave[b].x)[wid] = word;
        }
        __syncthreads();
        const int4 wv = s_wave[b];
        if ((wv.x | wv.y | wv.z | wv.w) & kLeanStop) return kFlagFar | kFlagReach;  // the same in every thread
        // the window: this wavefront's sources and its neighbours'
        const int wm = wid == 0 ? wv.x : (wid == 1 ? wv.y : (wid == 2 ? wv.z : wv.w));
        const int wl = wid == 0 ? wm : (wid == 1 ? wv.x : (wid == 2 ? wv.y : wv.z));
        const int wr = wid == 3 ? wm : (wid == 0 ? wv.y : (wid == 1 ? wv.z : wv.w));
        WaveInfo w;
        w.fxmin = min(lean_fxmin(wm), min(lean_fxmin(wl), lean_fxmin(wr)));
        w.fxmax = max(lean_fxmax(wm), max(lean_fxmax(wl), lean_fxmax(wr)));
        w.c1min = min(lean_c1min(wm), min(lean_c1min(wl), lean_c1min(wr)));
        w.c1max = max(lean_c1max(wm), max(lean_c1max(wl), lean_c1max(wr)));
        const bool fits_x = w.fxmin - (w.c1max + 1) >= -kMH && w.fxmax + 1 + (w.c1max + 1) <= kMH;
        const bool cmix = w.c1max == w.c1min + 1, xmix = w.fxmax == w.fxmin + 1;
        const bool fastw = fits_x && (w.c1max == w.c1min || cmix) && (w.fxmax == w.fxmin || xmix) && !(cmix && xmix);
        // FP32 storage: the row path (as the short pass takes them) for the
        // windows that mix both, or span three values of floor(v_x): at rest,
        // FP32 rounding leaves v_x a hair either side of 0.  In FP64 such
        // windows are rare, and the row path's registers would cost the pass
        // its occupancy: it gives those tiles up.
        constexpr bool kRows = sizeof(T) == 4;
        const bool rowsw = kRows && !fastw && fits_x && w.fxmax - w.fxmin <= 2;
        if (!fastw && !rowsw) far = 1;  // given up at the next barrier
        if constexpr (kRows) {
            if (dest && rowsw)
                gather_rows<T, L, 0, REST, SP, false, true>(R, tid, f, w.fxmin, w.fxmax, w.c1min, w.c1max, false, rq);
        }
        if (dest && fastw) {
            const int fx0 = w.fxmax;
            const int sel = (xmix ? 8 : 0) + (cmix ? 4 : 0) + w.c1min;
            switch (sel) {
                case 0: gather_fast<T, L, 0, 0, 2, 2, true, REST>(R, tid, fx0, f, rq); break;
                case 1: gather_fast<T, L, 0, 1, 2, 2, true, REST>(R, tid, fx0, f, rq); break;
                case 4: gather_fast<T, L, 0, 0, 3, 2, true, REST>(R, tid, fx0, f, rq); break;
                case 8: gather_fast<T, L, 0, 0, 2, 3, true, REST>(R, tid, fx0, f, rq); break;
                case 9: gather_fast<T, L, 0, 1, 2, 3, true, REST>(R, tid, fx0, f, rq); break;
                default: break;  // not reached: c'_1 <= 1, and cmix excludes xmix
            }
        }
        if (r >= 2 * L && dest) {
            T* __restrict__ orow = Yn + (Y0 + r - 2 * L) * nx;  // wave-uniform
            const T py = f.py0();
            at_byte(orow, gxb) = (T)f.a[0][kR];
            at_byte(orow + nn, gxb) = (T)f.a[0][kPx];
            at_byte(orow + 2 * nn, gxb) = py;
            at_byte(orow + 3 * nn, gxb) = (T)f.a[0][kE];
            tot[0] += (double)f.a[0][kR];
            tot[1] += (double)f.a[0][kPx];
            tot[2] += (double)py;
            tot[3] += (double)f.a[0][kE];
            if constexpr (SP) {
                at_byte(orow + 4 * nn, gxb) = (T)f.x[0];
                tot[NF - 1] += (double)f.x[0];
            }
        }
        f.shift();
    }
    // the last row's window decision has no later barrier to ride on
    __shared__ double s_sum[kMNW][NF];
    __shared__ int s_ir[kMNW][2];
#pragma unroll
    for (int c = 0; c < NF; ++c) tot[c] = wave_sum(tot[c]);
    reach = wave_max(reach);
    if (lane64 == 0) {
#pragma unroll
        for (int c = 0; c < NF; ++c) s_sum[wid][c] = tot[c];
        s_ir[wid][0] = reach;
        s_ir[wid][1] = far;
    }
    __syncthreads();
    int stop = 0;
#pragma unroll
    for (int w = 0; w < kMNW; ++w) stop |= s_ir[w][1];
    if (stop) return kFlagFar | kFlagReach;
    if (tid == 0) {
        int rr = 0;
        for (int c = 0; c < NF; ++c) {
            double t = s_sum[0][c];
            for (int w = 1; w < kMNW; ++w) t += s_sum[w][c];
            prow[c < 4 ? c : 6] = t;
        }
        for (int w = 0; w < kMNW; ++w) rr = max(rr, s_ir[w][0]);
        prow[4] = (double)rr;
        prow[5] = (double)(rr > kMH ? kErrReach : 0);
    }
    return 0;
}

// Wavefronts per SIMD the kernels are compiled for.  Short pass: FP64 keeps
// its FIFO in registers at two; FP32 fits four with a few spilled registers.
// Lean pass: four in FP64 (its 5-slot FIFO and one staged row per barrier
// leave the registers and LDS for them), more in FP32.
#ifndef LB_MARCH_WPE
#define LB_MARCH_WPE 2
#endif
#ifndef LB_MARCH_WPE_F32
#define LB_MARCH_WPE_F32 3
#endif
#ifndef LB_MARCH_WPE_FULL
#define LB_MARCH_WPE_FULL 1
#endif
#ifndef LB_LEAN_WPE
#define LB_LEAN_WPE 4
#endif
#ifndef LB_LEAN_WPE_F32
#define LB_LEAN_WPE_F32 4
#endif
#ifndef LB_LEAN_WPE_EXT
#define LB_LEAN_WPE_EXT 3  // FP64 with a rest level or two gases: more packets or fields per source
#endif

// Counters of StepCtl::next / PoolView::next: tile claims of each pass, and
// the tiles the lean and short passes left to the next pass (reset by the
// step's reduction kernel).
enum { kNextShort = 0, kNextFull = 1, kNextShortFlagged = 2, kNextLean = 3, kNextLeanFlagged = 4 };

// The lean pass (first of a step): persistent blocks claim the tiles (tiles_x
// column strips x row chunks of sy rows, row chunk major).  A tile it
// completes gets flags[t] = 0 (no bit of the short or full pass); one it
// gives up gets kFlagFar | kFlagReach in flags_lean[t], and flags[t] is left
// for the short pass (a kFlagKeep bit there from the previous step's full
// pass still counts).
template <typename T, bool WALLS, bool REST, bool SP>
__global__ void __launch_bounds__(kMTPB) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? LB_LEAN_WPE_F32 : ((REST || SP) ? LB_LEAN_WPE_EXT : LB_LEAN_WPE))))
march2d_lean_kernel(const T* __restrict__ Y, T* __restrict__ Yn, Grid g, Consts k, StepCtl* __restrict__ ctl,
                    double* __restrict__ partials, int* __restrict__ flags, int* __restrict__ flags_lean,
                    long long step, int sy, int tiles_x, int ntiles, int split)
{
    __shared__ int s_t;
    if (ctl->err_step < step) return;
    for (;;) {
        const int t = claim_tile(&ctl->next[kNextLean], &s_t);
        if (t >= ntiles) break;
        if (flags_lean[t] & kFlagKeep) {  // the short pass found it beyond this pass last step
            if (threadIdx.x == 0) {
                flags_lean[t] = kFlagFar | kFlagReach | kFlagKeep;
                atomicAdd(&ctl->next[kNextLeanFlagged], 1);
                if (split) flags[(2 + (step & 1)) * (int64_t)ntiles + t] = 0;
            }
            continue;
        }
        const int64_t tx = t % tiles_x, ty = t / tiles_x;
        const int bits = march_tile_lean<T, WALLS, REST, SP>(Y, Yn, g, k, tx * (kMTPB - 2 * kMH), ty * sy, sy,
                                                             partials + (int64_t)t * kPartialStride);
        if (threadIdx.x == 0) {
            flags_lean[t] = bits;
            if (bits) {
                atomicAdd(&ctl->next[kNextLeanFlagged], 1);
            } else {
                flags[t] = 0;
            }
            // the work word of this step starts clear (the short and full
            // passes set it for the tiles they compute)
            if (split) flags[(2 + (step & 1)) * (int64_t)ntiles + t] = 0;
        }
    }
}

// L = kLSmall: the short-FIFO pass over the tiles the lean pass gave up and
// their row-chunk neighbours (needs_pass on the lean pass's flags); it flags
// those it cannot complete itself.  L = kLFull: computes the tiles the short
// pass flagged and their neighbours (bit-identically: the summation order
// does not depend on L) and keeps the flag of each that still needs the full
// FIFO; the next step's short pass leaves such tiles to the full pass instead
// of computing them twice (flows change little per step).  Each returns at
// once when the previous pass flagged nothing.  With split (flags then holds
// the split state after its two words per tile, march2d_flag_bytes), a
// block claims a row chunk of a tile at a time (see kSplitMax).
template <typename T, int L, bool WALLS, bool REST, bool SP>
__global__ void __launch_bounds__(kMTPB) __attribute__((amdgpu_waves_per_eu(L < kLFull ? (sizeof(T) == 4 ? LB_MARCH_WPE_F32 : LB_MARCH_WPE) : LB_MARCH_WPE_FULL)))
march2d_kernel(const T* __restrict__ Y, T* __restrict__ Yn, Grid g, Consts k,
               StepCtl* __restrict__ ctl, double* __restrict__ partials, int* __restrict__ flags,
               int* __restrict__ flags_lean, long long step, int sy, int tiles_x, int ntiles, int split)
{
    __shared__ int s_t;
    if (ctl->err_step < step) return;
    const int nflag = ctl->next[L < kLFull ? kNextLeanFlagged : kNextShortFlagged];
    if (nflag == 0) return;  // nothing left to it
    // some tile kept its flag in the previous step's full pass (else no flag
    // holds kFlagKeep and the short pass need not look)
    const bool kept = L < kLFull && ctl->keep[1] != 0;
    // row chunks (see kSplitMax): work measured in the previous step and its
    // list of tiles to cut, work and list of this step, finished chunks per
    // tile, per-chunk partial slots
    const int nsx = split ? kSplitMax : 1;
    const int* __restrict__ work_in = flags + (2 + ((step - 1) & 1)) * (int64_t)ntiles;
    int* __restrict__ work_out = flags + (2 + (step & 1)) * (int64_t)ntiles;
    int* __restrict__ done = flags + 4 * (int64_t)ntiles;
    const int* __restrict__ list_in = flags + (5 + ((step - 1) & 1)) * (int64_t)ntiles;
    int* __restrict__ list_out = flags + (5 + (step & 1)) * (int64_t)ntiles;
    int* __restrict__ full_list = flags + 7 * (int64_t)ntiles;
    double* __restrict__ slots = reinterpret_cast<double*>(flags + split_slots_offset(ntiles));
    // the short pass cuts the listed tiles (by their work); the full pass
    // takes the tiles the short pass listed for it (each flagged tile and
    // the row chunks within two of one whose sources reach far: a superset
    // of those needs_pass selects) and cuts them all alike
    const int nlist = (L < kLFull && split) ? ctl->split_n[(step - 1) & 1] : 0;
    const int nfull = (L == kLFull && split) ? ctl->full_n : 0;
    const int ns_full = min(nsx, max(1, (int)gridDim.x / max(1, nfull)));
    const int nclaim = L < kLFull ? nlist * nsx + ntiles : (split ? nfull * nsx : ntiles);
    // short pass with row chunks: list tile tq for the full pass, once
    auto list_full = [&](int64_t tq) {
        if (!(atomicOr(&flags_lean[tq], kFlagFullListed) & kFlagFullListed))
            full_list[atomicAdd(&ctl->full_n, 1)] = (int)tq;
    };
    // ... a tile with flag bits fb: itself if flagged, and the row chunks
    // within two of it (same column strip, wrapped when y is periodic) if its
    // sources reach far (those whose halo rows it may own)
    auto list_for_full = [&](int64_t tq, int fb) {
        if (fb & kFlagFar) list_full(tq);
        if (fb & kFlagReach) {
            const int64_t chunks = ntiles / tiles_x, cx = tq % tiles_x, cy = tq / tiles_x;
            for (int d = -2; d <= 2; ++d) {
                int64_t y2 = cy + d;
                if (g.bc_y == kBcPeriodic) y2 = (y2 % chunks + chunks) % chunks;
                else if (y2 < 0 || y2 >= chunks) continue;
                list_full(y2 * tiles_x + cx);
            }
        }
    };
    auto chunks_of = [&](int t) -> int {
        if (nsx == 1) return 1;
        if (L == kLFull) return ns_full;
        return min(nsx, 1 + (work_in[t] & ~kWorkListed) / kSplitWork);
    };
    for (;;) {
        const int c = claim_tile(&ctl->next[L < kLFull ? kNextShort : kNextFull], &s_t);
        if (c >= nclaim) break;
        // short pass: the chunks of the listed tiles (they start with the
        // pass), then every tile not cut; full pass: nsx rounds over the
        // tiles, round q taking chunk q of each.  Other claims are skipped at once.
        int t, q;
        if (L < kLFull) {
            const bool listed = c < nlist * nsx;
            t = listed ? list_in[c / nsx] : c - nlist * nsx;
            q = listed ? c % nsx : -1;
        } else if (split) {
            t = full_list[c / nsx];
            q = c % nsx;
        } else {
            q = 0;
            t = c;
        }
        const int64_t tx = t % tiles_x, ty = t / tiles_x;
        const int64_t Y0 = ty * sy, ylast = min(Y0 + sy, g.ny);
        const int rows = (int)(ylast - Y0);
        int ns = chunks_of(t);
        const int h = (rows + ns - 1) / ns;  // rows per chunk; the last may be shorter
        ns = (rows + h - 1) / h;             // chunks with rows
        int p = 0;
        if (L < kLFull) {
            if (ns > 1 ? (q < 0 || q >= ns) : q >= 0) continue;  // cut: its chunks' claims; whole: its own
            p = ns > 1 ? q : 0;
        } else {
            if (ns > 1 ? q >= ns : q != 0) continue;
            p = q;
        }
        if (L < kLFull) {
            if (!needs_pass<kLLean>(flags_lean, 0, tiles_x, tx, Y0, ylast, sy, g.ny, g.bc_y)) continue;
            if (kept && (flags[t] & kFlagKeep)) {  // needed the full pass last step: left to it
                if (p == 0 && threadIdx.x == 0) {
                    flags[t] = kFlagFar | kFlagReach | kFlagKeep;
                    atomicAdd(&ctl->next[kNextShortFlagged], 1);
                    if (split) list_for_full(t, kFlagFar | kFlagReach);
                }
                continue;
            }
        } else if (!needs_pass<kLSmall>(flags, 0, tiles_x, tx, Y0, ylast, sy, g.ny, g.bc_y)) {
            continue;
        }
        const int64_t c0 = Y0 + (int64_t)p * h;
        const int hc = (int)min((int64_t)h, ylast - c0);
        double* const prow = ns > 1 ? slots + ((int64_t)p * ntiles + t) * kPartialStride
                                    : partials + (int64_t)t * kPartialStride;
        int work = 0;
        const int bits = march_tile<T, L, WALLS, REST, SP>(Y, Yn, g, k, tx * (kMTPB - 2 * kMH), c0, hc, prow, &work);
        if (threadIdx.x == 0) {
            int tb = bits, tw = work;
            bool last = true;
            if (ns > 1) {
                // this chunk's flag bits and work beside its sums; count it in,
                // and the last chunk adds the slots in chunk order
                prow[7] = (double)(work * 16 + bits);
                __threadfence();
                last = atomicAdd(&done[t], 1) == ns - 1;
                if (last) {
                    __threadfence();
                    done[t] = 0;
                    double sum[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
                    int rr = 0, ee = 0;
                    tb = 0;
                    tw = 0;
                    for (int i = 0; i < ns; ++i) {
                        const double* sr = slots + ((int64_t)i * ntiles + t) * kPartialStride;
                        double v[8];
#pragma unroll
                        for (int f = 0; f < 8; ++f)
                            v[f] = __hip_atomic_load(sr + f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                        for (int f = 0; f < 4; ++f) sum[f] += v[f];
                        sum[4] += v[6];
                        rr = max(rr, (int)v[4]);
                        ee |= (int)v[5];
                        const int wb = (int)v[7];
                        tb |= wb & 15;
                        tw += wb >> 4;
                    }
                    double* const row = partials + (int64_t)t * kPartialStride;
#pragma unroll
                    for (int f = 0; f < 4; ++f) row[f] = sum[f];
                    row[4] = (double)rr;
                    row[5] = (double)ee;
                    row[6] = sum[4];
                    // the chunks' work over the rows of one whole tile
                    tw = (int)((int64_t)tw * (rows + 2 * L) / (rows + ns * 2 * L));
                }
            }
            if (last) {
                const int far = tb & kFlagFar;
                if (L < kLFull) {
                    flags[t] = tb & (kFlagFar | kFlagReach);
                    if (far) atomicAdd(&ctl->next[kNextShortFlagged], 1);
                    // keep the lean pass's bits, which other blocks of this
                    // pass read, and the full pass's list mark, which they set
                    atomicAnd(&flags_lean[t], kFlagFar | kFlagReach | kFlagFullListed);
                    if (tb & kFlagNotLean) atomicOr(&flags_lean[t], kFlagKeep);
                    if (split) list_for_full(t, tb);
                } else {
                    // keep the short pass's bits, which other blocks of this pass read
                    flags[t] = (flags[t] & (kFlagFar | kFlagReach)) | (far ? kFlagKeep : 0);
                    atomicAdd(&ctl->redo_tiles, 1);
                    if (far) atomicAdd(&ctl->keep[0], 1);
                }
                if (nsx > 1) {
                    // this step's work; a tile worth cutting is listed once
                    const int was = work_out[t];
                    const bool list = tw >= kSplitWork && !(was & kWorkListed);
                    work_out[t] = min(tw, kWorkListed - 1) | ((list || (was & kWorkListed)) ? kWorkListed : 0);
                    if (list) list_out[atomicAdd(&ctl->split_n[step & 1], 1)] = t;
                }
            }
        }
    }
}

// Pool form of the three passes: persistent blocks claim tiles of the tile
// table (see pool1d_kernel); a slot's tiles are its row chunks, then column
// strips, from its t0, which is how needs_pass finds a tile's neighbours.
template <typename T, bool WALLS, bool REST, bool SP>
__global__ void __launch_bounds__(kMTPB) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? LB_LEAN_WPE_F32 : ((REST || SP) ? LB_LEAN_WPE_EXT : LB_LEAN_WPE))))
pool2d_lean_kernel(PoolView v, Consts k)
{
    __shared__ int s_t;
    const int nt = *v.ntiles;
    T* arena = (T*)v.arena;
    for (;;) {
        const int t = claim_tile(&v.next[kNextLean], &s_t);
        if (t >= nt) break;
        const int ts = v.tstate[t];
        if (!(ts & kTileLive)) continue;  // the same for the whole block
        if (v.flags_lean[t] & kFlagKeep) {  // the short pass found it beyond this pass last step
            if (threadIdx.x == 0) {
                v.flags_lean[t] = kFlagFar | kFlagReach | kFlagKeep;
                atomicAdd(&v.next[kNextLeanFlagged], 1);
            }
            continue;
        }
        const PoolTile& tl = v.tiles[t];
        const int64_t o0 = tl.off[0], o1 = tl.off[1];
        const int64_t from = (ts & kTileSet) ? o1 : o0, to = (ts & kTileSet) ? o0 : o1;
        const Grid g{tl.nx, tl.ny, tl.bc_x, tl.bc_y};
        const int bits = march_tile_lean<T, WALLS, REST, SP>(arena + from, arena + to, g, k, tl.x0, tl.y0,
                                                             tl.rows, v.partials + (int64_t)t * kPartialStride);
        if (threadIdx.x == 0) {
            v.flags_lean[t] = bits;
            if (bits) atomicAdd(&v.next[kNextLeanFlagged], 1);
            else v.flags[t] = 0;
        }
    }
}

template <typename T, int L, bool WALLS, bool REST, bool SP>
__global__ void __launch_bounds__(kMTPB) __attribute__((amdgpu_waves_per_eu(L < kLFull ? (sizeof(T) == 4 ? LB_MARCH_WPE_F32 : LB_MARCH_WPE) : LB_MARCH_WPE_FULL)))
pool2d_kernel(PoolView v, Consts k)
{
    __shared__ int s_t;
    if (v.next[L < kLFull ? kNextLeanFlagged : kNextShortFlagged] == 0) return;  // nothing left to it
    const int nt = *v.ntiles;
    T* arena = (T*)v.arena;
    for (;;) {
        const int t = claim_tile(&v.next[L < kLFull ? kNextShort : kNextFull], &s_t);
        if (t >= nt) break;
        const int ts = v.tstate[t];
        if (!(ts & kTileLive)) continue;  // the same for the whole block
        const PoolTile& tl = v.tiles[t];
        const int64_t tiles_x = (tl.nx + kPool2Cols - 1) / kPool2Cols;
        const int64_t tbase = v.probs[tl.prob].t0, tx = tl.x0 / kPool2Cols;
        const int64_t ylast = min(tl.y0 + (int64_t)tl.rows, tl.ny);
        if (L < kLFull) {
            if (!needs_pass<kLLean>(v.flags_lean, tbase, tiles_x, tx, tl.y0, ylast, tl.rows, tl.ny, tl.bc_y))
                continue;
            if (v.flags[t] & kFlagKeep) {  // needed the full FIFO last step: left to the full pass
                if (threadIdx.x == 0) {
                    v.flags[t] = kFlagFar | kFlagReach | kFlagKeep;
                    atomicAdd(&v.next[kNextShortFlagged], 1);
                }
                continue;
            }
        } else if (!needs_pass<kLSmall>(v.flags, tbase, tiles_x, tx, tl.y0, ylast, tl.rows, tl.ny, tl.bc_y)) {
            continue;
        }
        const int64_t o0 = tl.off[0], o1 = tl.off[1];  // selected below, not indexed (keeps them in registers)
        const int64_t from = (ts & kTileSet) ? o1 : o0, to = (ts & kTileSet) ? o0 : o1;
        const Grid g{tl.nx, tl.ny, tl.bc_x, tl.bc_y};
        const int bits = march_tile<T, L, WALLS, REST, SP>(arena + from, arena + to, g, k, tl.x0, tl.y0, tl.rows,
                                                           v.partials + (int64_t)t * kPartialStride);
        if (threadIdx.x == 0) {
            const int far = bits & kFlagFar;
            if (L < kLFull) {
                v.flags[t] = bits & (kFlagFar | kFlagReach);
                if (far) atomicAdd(&v.next[kNextShortFlagged], 1);
                // keep the lean pass's bits, which other blocks of this pass read
                v.flags_lean[t] = (v.flags_lean[t] & (kFlagFar | kFlagReach)) |
                                  ((bits & kFlagNotLean) ? kFlagKeep : 0);
            } else {
                // keep the short pass's bits, which other blocks of this pass read
                v.flags[t] = (v.flags[t] & (kFlagFar | kFlagReach)) | (far ? kFlagKeep : 0);
            }
        }
    }
}

// The three passes of one step: lean over every tile, short over what the
// lean pass gave up (and its neighbours), full over what the short pass
// flagged (and its neighbours).  nblocks_lean persistent blocks for the lean
// pass, m.nblocks for the others.  flags holds 2 ntiles ints: the short and
// full passes' flags, then the lean pass's.
template <typename T, bool WALLS, bool REST, bool SP>
hipError_t launch_march2d_w(const T* Y, T* Yn, const Grid& g, const MarchGeom& m, const Consts& k,
                            StepCtl* ctl, double* partials, int* flags, long long step, hipStream_t stream,
                            bool split)
{
    const int nt = (int)m.blocks();
    int* flags_lean = flags + nt;
    const int sp = split ? 1 : 0;
    march2d_lean_kernel<T, WALLS, REST, SP><<<m.nblocks_lean, kMTPB, 0, stream>>>(
        Y, Yn, g, k, ctl, partials, flags, flags_lean, step, m.sy, (int)m.grid_x, nt, sp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    march2d_kernel<T, kLSmall, WALLS, REST, SP><<<m.nblocks, kMTPB, 0, stream>>>(
        Y, Yn, g, k, ctl, partials, flags, flags_lean, step, m.sy, (int)m.grid_x, nt, sp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    march2d_kernel<T, kLFull, WALLS, REST, SP><<<m.nblocks, kMTPB, 0, stream>>>(
        Y, Yn, g, k, ctl, partials, flags, flags_lean, step, m.sy, (int)m.grid_x, nt, sp);
    return hipGetLastError();
}

// The three passes of one pool step.
template <typename T, bool WALLS, bool REST, bool SP>
hipError_t launch_pool2d_w(const PoolView& v, const Consts& k, int nblocks_lean, int nblocks, hipStream_t stream)
{
    pool2d_lean_kernel<T, WALLS, REST, SP><<<nblocks_lean, kMTPB, 0, stream>>>(v, k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    pool2d_kernel<T, kLSmall, WALLS, REST, SP><<<nblocks, kMTPB, 0, stream>>>(v, k);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    pool2d_kernel<T, kLFull, WALLS, REST, SP><<<nblocks, kMTPB, 0, stream>>>(v, k);
    return hipGetLastError();
}

}  // namespace

// Two gases (lb_march2d_sp.hip, lb_pool2d_sp.hip): the instances with the
// species field.
template <typename T>
hipError_t launch_march2d_species(const T* Y, T* Yn, const Grid& g, const MarchGeom& m, const Consts& k,
                                  StepCtl* ctl, double* partials, int* flags, long long step,
                                  hipStream_t stream, bool split);
template <typename T>
hipError_t launch_pool2d_species(const PoolView& v, const Consts& k, int nblocks_lean, int nblocks, bool walls,
                                 hipStream_t stream);

}  // namespace lbsd
