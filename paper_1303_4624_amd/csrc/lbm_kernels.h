// lbm_kernels.h - HIP kernels for CDNA4 (gfx950) of the thermal lattice
// Boltzmann update with the on-lattice models (D2Q33, D3Q95 of 4th order;
// the lower-order D3Q19, D3Q15), and the launchers of one model and
// precision (ModelKernels<M, P>).  Included only by the lbm_kernels_*.hip
// translation units, each of which instantiates the launchers of one model
// (and precision), so that the models compile in parallel.
//
// Data layout: row-blocked.  The Q populations of a group of consecutive
// grid rows are contiguous, population-major (see PopAt / row_base), cells
// x-fastest.  One thread owns one cell and a block one grid row (or a chunk
// of it, or several whole rows of 64j cells).  Every population read is a contiguous run of a source row
// (neighbouring threads read neighbouring x), so the gather f_i(x - e_i) is
// coalesced; the x-wrap of the periodic grid is folded into a per-lane
// offset, the y/z-wrap into wave-uniform slab bases and row offsets.
//
// Precision variants:
//   F64  : f_i stored and computed in float64.
//   F32S : g_i = f_i - w_i rho0 stored in float32.  The moment sums are
//          accumulated in float64; the per-cell scalars (rho, U, theta) and
//          the per-group coefficients are formed in float64 and rounded once
//          per cell; the polynomial, relaxation and store are float32.
//          Rounding the model constants themselves to float32 would change
//          the model by ~1e-8 in every cell and step alike; per-cell rounding
//          only adds noise.  The O(1) part w_i rho0 never enters float32
//          arithmetic.
//
// Streaming: two buffers (k_step: pull from one, store to the other) or one
// buffer updated in place (k_step_aa, the AA pattern).
//
// Equilibrium: the Hermite expansion of the Maxwellian of order N (N = 4 for
// the 4th-order models, N = 2 for the 2nd-order ones), written as a
// polynomial in s = xi_i . u_hat for each symmetry group (|e_i|^2 is
// constant on a group, so every coefficient except s is per group):
//   N = 4:  P_i = 1 + h_i,  h_i = a0 + s (a1 + s (a2 + s (1/6 + s/24)))
//   a0 = (-u2 + d (X - D)) / 2
//        + (3 u2^2 + 6 d (D + 2 - X) u2 + 3 d^2 (X^2 - 2 (D + 2) X + D (D + 2))) / 24
//   a1 = 1 - u2/2 + d (X - D - 2)/2,   a2 = 1/2 - u2/4 + d (X - D - 4)/4
//   N = 2:  h_i = (-u2 + d (X - D)) / 2 + s (1 + s/2)
// with xi_i = e_i / c_s, c_s^2 = T0, u_hat = U / c_s, u2 = |u_hat|^2,
// X = |xi_i|^2 and d = T/T0 - 1, so s = e_i . U / T0.  This is the
// contraction of sum_{n<=N} a^(n):H^(n)(xi)/n! with the Hermite coefficients
// of the Maxwellian, collected in powers of s.  Per cell the coefficients
// are formed once as polynomials in X (XPoly); per group only X_g enters.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "lbm_internal.h"

namespace lbm {
namespace {

// Build-time switches, each at its measured best (alternatives timed on the
// same buffers unless noted):
// non-temporal stores of the two-buffer steps (plain stores 4-8 % slower);
#ifndef LBM_NT_STORE
#define LBM_NT_STORE 1
#endif
// non-temporal loads (8 % slower);
#ifndef LBM_NT_LOAD
#define LBM_NT_LOAD 0
#endif
// each XCD takes a contiguous range of rows (round-robin 4-5 % slower);
#ifndef LBM_XCD_REMAP
#define LBM_XCD_REMAP 1
#endif
// occupancy target of the FP32-shifted adjoint kernel (waves per SIMD): 3
// waves (<= 168 VGPRs) fit without scratch when its loads are issued in
// velocity order (LBM_ADJ_GATHER_SORTED 0); sorted by source row they need
// about 180 VGPRs, which fit 2 waves only;
#ifndef LBM_ADJ_WAVES
#define LBM_ADJ_WAVES 3
#endif
// minimum waves per SIMD of the FP32-shifted steps (the compiler's budget;
// they hold 125-172 VGPRs);
#ifndef LBM_F32_WAVES
#define LBM_F32_WAVES 1
#endif
// the pushed stores of the AA kernel start at x + e_x, off the 128-byte line
// grid; plain stores let L2 merge the partial lines of neighbouring waves
// before they reach HBM (non-temporal 8 % slower); its own-row stores are
// non-temporal like the two-buffer step's;
#ifndef LBM_AA_NT_PUSH
#define LBM_AA_NT_PUSH 0
#endif
#ifndef LBM_AA_NT_LOCAL
#define LBM_AA_NT_LOCAL 1
#endif
// float64 moment sums of the FP32-shifted storage (see F32ST).
#ifndef LBM_F32S_SUM64
#define LBM_F32S_SUM64 1
#endif
constexpr int kBlock = 256;            // threads per block of the cell-parallel kernels
constexpr int kW = 2 * kMaxDisp + 1;   // distinct displacement components

template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(static_cast<F&&>(f), std::make_integer_sequence<int, N>{});
}

// Storage precisions (their block limits: row_block_limit).
struct F64T {
    using S = double;
    using Acc = double;   // type of the per-cell moment sums
    static constexpr Prec id = Prec::F64;
    static constexpr bool shifted = false;
    static constexpr int waves = 1;
    static constexpr int adj_waves = 1;
};
struct F32ST {
    using S = float;
    static constexpr Prec id = Prec::F32S;
    // Moment sums of the float32 deviations in float64: a float32 sum of 95
    // terms is off by a few ulps of sum |e|^2 |g|, the same in every node of
    // a uniform region, so without it such regions drift coherently.
#if LBM_F32S_SUM64
    using Acc = double;
#else
    using Acc = float;
#endif
    static constexpr bool shifted = true;
    static constexpr int waves = LBM_F32_WAVES;
    static constexpr int adj_waves = LBM_ADJ_WAVES;
};

template <Prec P>
struct PrecOf {
    using type = F64T;
};
template <>
struct PrecOf<Prec::F32S> {
    using type = F32ST;
};

// (v mod n) for v in [-kMaxDisp, n - 1 + kMaxDisp]; n is wave-uniform.
__device__ __forceinline__ int wrap_idx(int v, int n) {
    if (n > kMaxDisp) {
        v += (v < 0) ? n : 0;
        v -= (v >= n) ? n : 0;
        return v;
    }
    v %= n;
    return v < 0 ? v + n : v;
}

struct Cell {
    int x, y, z;        // x clamped into the grid for inactive lanes
    int row;            // y + ny*z
    bool active;
    long long c;        // linear cell index
};

// Storage layout of the populations: the Q populations of a group of rg
// consecutive grid rows (fixed z; rg = 1 in 2D) are contiguous,
// population-major, the rg rows of one population adjacent: population i
// of cell (x, y, z) sits at row_base(y, z) + i*rg*rs + x, rs >= nx the run
// stride (KParams::rs, KParams::rg).  A step then writes contiguous runs per
// row and reads Q runs from the few source rows around it.
//
// Where population i of cell c is stored depends on the form of the state
// (KParams::form): kFormAB, run i of cell c; kFormSwapped (in-place AA
// pattern after an even number of steps), run opp(i) of cell c;
// kFormPushed (AA after an odd number), run i of cell c + e_i.
// Element offset of the first population run of grid row (y, z): rows are
// taken in groups of rg consecutive y (same z) whose runs interleave, so a
// population run of a group is rg*rs elements long.
__device__ __forceinline__ long long row_base(const KParams& k, int Q, int y, int z) {
    const int gy = y >> k.rg_shift;
    const int ry = y - (gy << k.rg_shift);
    return (static_cast<long long>(z) * k.ny * Q + static_cast<long long>(gy) * Q * k.rg + ry) *
           k.rs;
}

// Element index of population i of cell c in storage form FORM (a
// compile-time copy of KParams::form, see with_form).  The per-cell work
// (divisions, and the neighbour offsets of the pushed form) is done once in
// the constructor; at<i>() is a few adds.  Cell indices fit in 32 bits
// (N < 2^31 is checked on the host).
__device__ __forceinline__ void cell_xyz(const KParams& k, long long c, int& x, int& y, int& z) {
    const unsigned cu = static_cast<unsigned>(c);
    const unsigned row = cu / static_cast<unsigned>(k.nx);
    x = static_cast<int>(cu - row * static_cast<unsigned>(k.nx));
    y = static_cast<int>(row % static_cast<unsigned>(k.ny));
    z = static_cast<int>(row / static_cast<unsigned>(k.ny));
}

template <class M, int FORM>
struct PopAt {
    long long base;              // own cell, run 0
    long long pstride;           // elements between two population runs
    __device__ __forceinline__ PopAt(const KParams& k, long long c) {
        int x, y, z;
        cell_xyz(k, c, x, y, z);
        pstride = static_cast<long long>(k.rg) * k.rs;
        base = row_base(k, M::Q, y, z) + x;
    }
    template <int i>
    __device__ __forceinline__ long long at() const {
        constexpr int slot = (FORM == kFormSwapped) ? M::table.opp[i] : i;
        return base + slot * pstride;
    }
};

template <class M>
struct PopAt<M, kFormPushed> {
    long long pstride;
    long long zo[kW], yo[kW];    // row offsets of the cells at +d
    int xo[kW];
    __device__ __forceinline__ PopAt(const KParams& k, long long c) {
        int x, y, z;
        cell_xyz(k, c, x, y, z);
        pstride = static_cast<long long>(k.rg) * k.rs;
        static_for<kW>([&](auto DI) {
            constexpr int d = decltype(DI)::value - kMaxDisp;
            xo[d + kMaxDisp] = wrap_idx(x + d, k.nx);
            yo[d + kMaxDisp] = row_base(k, M::Q, wrap_idx(y + d, k.ny), 0);
            zo[d + kMaxDisp] =
                (M::D == 3) ? static_cast<long long>(wrap_idx(z + d, k.nz)) * k.ny * M::Q * k.rs : 0;
        });
    }
    template <int i>
    __device__ __forceinline__ long long at() const {
        constexpr int ex = M::table.e[i][0], ey = M::table.e[i][1], ez = M::table.e[i][2];
        return zo[ez + kMaxDisp] + yo[ey + kMaxDisp] + i * pstride + xo[ex + kMaxDisp];
    }
};

// Row-blocked mapping: block b covers threads [chunk*bx, chunk*bx + bx) of
// grid row `row` = y + ny*z.  y and z are uniform over the block.
// Blocks are dispatched round-robin over the 8 XCDs.  By default each XCD
// takes a contiguous range of rows, so the chunks of a row share one L2.
// CYCLIC (the forward steps, which sum nothing across blocks, so the mapping
// cannot change a result): with k.xcd_cyclic > 0 and a grid of a multiple of
// 8 * xcd_cyclic blocks, the XCDs take chunks of xcd_cyclic blocks in turn
// instead.  Which of the two is faster depends on where the buffers lie in
// HBM (lbm_tune_step measures it).
template <bool CYCLIC = false>
__device__ __forceinline__ Cell row_cell(const KParams& k) {
#if LBM_XCD_REMAP
    const int hb = blockIdx.x;
    const int nb = gridDim.x;
    const int xcd = hb & 7, pos = hb >> 3;
    const int cc = CYCLIC ? k.xcd_cyclic : 0;
    int b;
    if (cc > 0 && nb % (8 * cc) == 0) {
        b = ((pos / cc) * 8 + xcd) * cc + pos % cc;
    } else {
        const int q = nb >> 3, r = nb & 7;
        b = (xcd < r) ? xcd * (q + 1) + pos : r * (q + 1) + (xcd - r) * q + pos;
    }
#else
    const int b = blockIdx.x;
#endif
    int row, x;
    if (kPackRows && k.rpb > 1) {
        // rpb whole rows of nx (a multiple of 64) lanes: the row is uniform
        // over each wave
        const int sub = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / k.nx);
        row = b * k.rpb + sub;
        x = static_cast<int>(threadIdx.x) - sub * k.nx;
    } else {
        const int chunk = b % k.chunks;
        row = b / k.chunks;
        x = chunk * k.bx + static_cast<int>(threadIdx.x);
    }
    Cell cl;
    cl.active = x < k.nx;
    cl.x = cl.active ? x : 0;
    cl.row = row;
    cl.y = row % k.ny;
    cl.z = row / k.ny;
    cl.c = (static_cast<long long>(row)) * k.nx + cl.x;
    return cl;
}

// Addresses around one cell: a 64-bit base per slab of the slowest axis
// (z-planes in 3D, rows in 2D; wave-uniform) plus a 32-bit byte offset inside
// the slab (row, population run, x).  A slab stays below 4 GiB (checked on
// the host).  at<slot, dx, dy, dz>() is the address of population run `slot`
// of cell (x + dx, y + dy, z + dz), periodic; |d| <= kMaxDisp.
template <class M, class S, class B>
struct SlabAddr {
    unsigned runb;
    unsigned xb[kW], yb[kW];
    B* sb[kW];
    __device__ __forceinline__ SlabAddr(B* base, const KParams& k, const Cell& cl) {
        const unsigned rsb = static_cast<unsigned>(k.rs) * static_cast<unsigned>(sizeof(S));
        runb = rsb * static_cast<unsigned>(k.rg);
        const unsigned groupb = runb * static_cast<unsigned>(M::Q);   // one row group
        static_for<kW>([&](auto DI) {
            constexpr int d = decltype(DI)::value - kMaxDisp;   // table entry d: cell at -d
            xb[d + kMaxDisp] = static_cast<unsigned>(wrap_idx(cl.x - d, k.nx)) * sizeof(S);
            const int yr = wrap_idx(cl.y - d, k.ny);
            const int gy = yr >> k.rg_shift, ry = yr - (gy << k.rg_shift);
            const unsigned inslab = static_cast<unsigned>(gy) * groupb + static_cast<unsigned>(ry) * rsb;
            if constexpr (M::D == 3) {
                yb[d + kMaxDisp] = inslab;
                sb[d + kMaxDisp] = base + static_cast<unsigned long long>(wrap_idx(cl.z - d, k.nz)) *
                                              (static_cast<unsigned long long>(rsb) * M::Q * k.ny);
            } else {
                yb[d + kMaxDisp] = 0u;
                sb[d + kMaxDisp] = base + static_cast<unsigned long long>(gy) * groupb +
                                   static_cast<unsigned long long>(ry) * rsb;
            }
        });
    }
    template <int slot, int dx, int dy, int dz>
    __device__ __forceinline__ B* at() const {
        constexpr int ds = (M::D == 3) ? dz : dy;      // along the slab axis
        constexpr int dr = (M::D == 3) ? dy : 0;       // rows inside a slab
        const unsigned off = yb[kMaxDisp - dr] + static_cast<unsigned>(slot) * runb + xb[kMaxDisp - dx];
        return sb[kMaxDisp - ds] + off;
    }
};

template <class S>
__device__ __forceinline__ S load_pop(const char* p) {
#if LBM_NT_LOAD
    return __builtin_nontemporal_load(reinterpret_cast<const S*>(p));
#else
    return *reinterpret_cast<const S*>(p);
#endif
}

template <class S, bool NT = (LBM_NT_STORE != 0)>
__device__ __forceinline__ void store_pop(char* p, S val) {
    if constexpr (NT)
        __builtin_nontemporal_store(val, reinterpret_cast<S*>(p));
    else
        *reinterpret_cast<S*>(p) = val;
}

// Gather v_i = src_i(x - SIGN*e_i) with periodic wrap on every axis.
// Order in which a gather issues its loads: the velocity order, or sorted
// by source slab, then source row.  The order changes no value, only the
// issue order.  Measured with builds of both orders bound to the same
// buffers: the forward pull sorted is faster in 3D (D3Q95 FP64 256^3 by
// 2.2 %, FP32-shifted 128^3 to 384^3 by 0.2-0.5 %, D3Q19 by 0.2 %) and slower
// in 2D (D2Q33 8192^2 by 0.2-0.5 %); the adjoint sorted needs ~180 VGPRs
// (2 waves per SIMD) and in velocity order fits 3 waves, which is 2 % faster
// at 128^3 (the adjoint of 200 steps with recomputation: 117.2 against
// 119.6 ms).
#ifndef LBM_FWD_GATHER_SORTED_3D
#define LBM_FWD_GATHER_SORTED_3D 1
#endif
#ifndef LBM_ADJ_GATHER_SORTED
#define LBM_ADJ_GATHER_SORTED 0
#endif
template <class M, bool SORTED>
struct LoadOrder {
    struct Arr {
        int v[M::Q];
    };
    static constexpr Arr make() {
        Arr o{};
        for (int i = 0; i < M::Q; ++i) o.v[i] = i;
        if (SORTED) {
            const auto key = [](int i) {
                return (M::table.e[i][2] * 16 + M::table.e[i][1]) * 16 + M::table.e[i][0];
            };
            for (int a = 1; a < M::Q; ++a)
                for (int b = a; b > 0 && key(o.v[b]) < key(o.v[b - 1]); --b) {
                    const int t = o.v[b];
                    o.v[b] = o.v[b - 1];
                    o.v[b - 1] = t;
                }
        }
        return o;
    }
    static constexpr Arr order = make();
};

// SIGN = +1 is the pull of the forward update, SIGN = -1 the transposed
// (adjoint) streaming.
template <class M, int SIGN, class S>
__device__ __forceinline__ void gather(const S* __restrict__ src, const KParams& k, const Cell& cl,
                                       S (&v)[M::Q]) {
    const SlabAddr<M, S, const char> ad(reinterpret_cast<const char*>(src), k, cl);
    constexpr bool sorted = SIGN < 0 ? LBM_ADJ_GATHER_SORTED != 0
                                     : (M::D == 3 && LBM_FWD_GATHER_SORTED_3D != 0);
    static_for<M::Q>([&](auto I) {
        constexpr int i = LoadOrder<M, sorted>::order.v[decltype(I)::value];
        constexpr int ex = SIGN * M::table.e[i][0];
        constexpr int ey = SIGN * M::table.e[i][1];
        constexpr int ez = SIGN * M::table.e[i][2];
        v[i] = load_pop<S>(ad.template at<i, -ex, -ey, -ez>());
    });
}

// Writes the populations of a cell in increasing order through one running
// 64-bit pointer (row start + population run) and the cell's 32-bit byte
// offset inside the run.  Lanes past the end of a ragged row have x clamped
// to 0: they compute bit-identical values for cell (0, y, z) and store them
// there too, which keeps the stores free of per-store branches.
template <class S>
struct PlaneWriter {
    char* run;
    unsigned long long runb;
    unsigned off;
    __device__ __forceinline__ PlaneWriter(S* dst, const KParams& k, const Cell& cl, int Q)
        : run(reinterpret_cast<char*>(dst) +
              static_cast<unsigned long long>(row_base(k, Q, cl.y, cl.z)) * sizeof(S)),
          runb(static_cast<unsigned long long>(k.rs) * k.rg * sizeof(S)),
          off(static_cast<unsigned>(cl.x) * static_cast<unsigned>(sizeof(S))) {}
    __device__ __forceinline__ void put(S val) {
        store_pop<S>(run + off, val);
        run += runb;
    }
};


// Per-cell macroscopic values in float64 from the raw sums of the stored
// values: m0 = sum v, j = sum v e, en = sum v |e|^2.
struct Macro {
    double rho, dr, ux, uy, uz, usq, d, u2;
};

template <int D, bool SHIFTED>
__device__ __forceinline__ Macro macro_from_sums(const KParams& k, double m0, double jx, double jy,
                                                 double jz, double en) {
    Macro m;
    if constexpr (SHIFTED) {
        m.dr = m0;
        m.rho = k.rho0 + m0;
    } else {
        m.rho = m0;
        m.dr = 0.0;
    }
    const double inv = 1.0 / m.rho;
    m.ux = jx * inv;
    m.uy = jy * inv;
    m.uz = (D == 3) ? jz * inv : 0.0;
    m.usq = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
    const double invDT0 = k.invT0 * (1.0 / D);
    if constexpr (SHIFTED) {
        // rho D T = sum g|e|^2 + rho0 D T0 - rho |U|^2, so rho D T0 (theta - 1)
        // = en - D T0 dr - rho |U|^2: no cancellation against rho0.
        m.d = (en - D * k.T0 * m.dr - m.rho * m.usq) * inv * invDT0;
    } else {
        m.d = (en * inv - m.usq) * invDT0 - 1.0;
    }
    m.u2 = m.usq * k.invT0;
    return m;
}

// Coefficients of h in powers of s for one group (float64), from the
// per-cell polynomials in X = |xi|^2 of the Hermite expansion of order N:
//   N = 4: a0 = a00 + X (a01 + X a02), a1 = a10 + a11 X, a2 = a20 + a21 X
//          (the a0, a1, a2 of the file header expanded in X);
//   N = 2: a0 = a00 + X a01, a1 = 1, a2 = 1/2.
struct GCoef {
    double a0, a1, a2;
};
template <int D, int N>
struct XPoly {
    double a00, a01, a02, a10, a11, a20, a21;
    __device__ __forceinline__ XPoly(double u2, double d) {
        constexpr double Dd = D;
        if constexpr (N == 4) {
            a00 = -0.5 * u2 + 0.125 * u2 * u2 +
                  d * (-0.5 * Dd + u2 * (0.25 * (Dd + 2.0)) + d * (0.125 * Dd * (Dd + 2.0)));
            a01 = d * (0.5 - 0.25 * u2 - d * (0.25 * (Dd + 2.0)));
            a02 = 0.125 * d * d;
            a10 = 1.0 - 0.5 * u2 - d * (0.5 * (Dd + 2.0));
            a11 = 0.5 * d;
            a20 = 0.5 - 0.25 * u2 - d * (0.25 * (Dd + 4.0));
            a21 = 0.25 * d;
        } else {
            static_assert(N == 2, "equilibrium order 2 or 4");
            a00 = -0.5 * u2 - d * (0.5 * Dd);
            a01 = 0.5 * d;
            a02 = 0.0;
            a10 = 1.0;
            a11 = 0.0;
            a20 = 0.5;
            a21 = 0.0;
        }
    }
    __device__ __forceinline__ GCoef at(double X) const {
        GCoef c;
        if constexpr (N == 4) {
            c.a0 = a00 + X * (a01 + X * a02);
            c.a1 = a10 + a11 * X;
            c.a2 = a20 + a21 * X;
        } else {
            c.a0 = a00 + X * a01;
            c.a1 = 1.0;
            c.a2 = 0.5;
        }
        return c;
    }
};

// X_g = |e_g|^2 / T0 of group g.
template <class M, int g>
__device__ __forceinline__ double group_x(const KParams& k) {
    return k.X[g];
}

// h(s) of order N with the group's coefficients (a1, a2 unused for N = 2,
// where they are the constants 1 and 1/2).
template <int N, class R>
__device__ __forceinline__ R horner_h(R a0, R a1, R a2, R s) {
    if constexpr (N == 4)
        return fma(s, fma(s, fma(s, fma(s, R(1.0 / 24.0), R(1.0 / 6.0)), a2), a1), a0);
    else
        return fma(s, fma(s, R(0.5), R(1)), a0);
}

// s_i = e_i . ut with compile-time integer components.
template <int ex, int ey, int ez, class R>
__device__ __forceinline__ R edot(R ux, R uy, R uz) {
    R s = R(0);
    if constexpr (ex != 0) s = R(ex) * ux;
    if constexpr (ey != 0) s = (ex != 0) ? fma(R(ey), uy, s) : R(ey) * uy;
    if constexpr (ez != 0) s = (ex != 0 || ey != 0) ? fma(R(ez), uz, s) : R(ez) * uz;
    return s;
}

// Sum over a block of K doubles per thread; thread 0 calls store(q, sum_q).
template <int K, class Store>
__device__ __forceinline__ void block_sum_with(double (&v)[K], Store&& store) {
    static_for<K>([&](auto KI) {
        constexpr int q = decltype(KI)::value;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
    });
    __shared__ double sh[(1024 / 64) * K];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    if (lane == 0) {
        static_for<K>([&](auto KI) {
            constexpr int q = decltype(KI)::value;
            sh[wid * K + q] = v[q];
        });
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        static_for<K>([&](auto KI) {
            constexpr int q = decltype(KI)::value;
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += sh[w * K + q];
            store(q, s);
        });
    }
}

// Sum over a block of K doubles per thread; thread 0 writes (or adds to) out[0..K).
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* out, bool accumulate) {
    block_sum_with<K>(v, [&](int q, double s) { out[q] = accumulate ? out[q] + s : s; });
}

// ---------------------------------------------------------------------------
// f^eq(r, U, T) of one cell in storage form, computed in float64 and
// rounded once (Formula (3)); emit(I, value) receives population I::value in
// increasing order.
template <class M, class P, class Emit>
__device__ __forceinline__ void feq_cell(const KParams& k, double r, double ux, double uy,
                                         double uz, double T, Emit&& emit) {
    using S = typename P::S;
    const double d = T * k.invT0 - 1.0;
    const double u2 = (ux * ux + uy * uy + uz * uz) * k.invT0;
    const double utx = ux * k.invT0, uty = uy * k.invT0, utz = uz * k.invT0;
    const XPoly<M::D, M::N> xp(u2, d);
    static_for<M::G>([&](auto GI) {
        constexpr int g = decltype(GI)::value;
        const GCoef gc = xp.at(group_x<M, g>(k));
        const double w = k.W[g];
        static_for<M::table.gsize[g]>([&](auto JI) {
            constexpr int i = M::table.gstart[g] + decltype(JI)::value;
            constexpr int ex = M::table.e[i][0], ey = M::table.e[i][1], ez = M::table.e[i][2];
            const double h =
                horner_h<M::N>(gc.a0, gc.a1, gc.a2, edot<ex, ey, ez>(utx, uty, utz));
            if constexpr (P::shifted)
                emit(std::integral_constant<int, i>{}, S(w * (r - k.rho0) + w * r * h));
            else
                emit(std::integral_constant<int, i>{}, S(w * r * (1.0 + h)));
        });
    });
}

// Store f^eq(r, U, T) of cell c in storage form FORM.
template <class M, class P, int FORM>
__device__ __forceinline__ void store_feq(typename P::S* __restrict__ f, const KParams& k,
                                          long long c, double r, double ux, double uy,
                                          double uz, double T) {
    const PopAt<M, FORM> pa(k, c);
    feq_cell<M, P>(k, r, ux, uy, uz, T, [&](auto I, typename P::S val) {
        f[pa.template at<decltype(I)::value>()] = val;
    });
}

// ---------------------------------------------------------------------------
// Moments, equilibrium and BGK relaxation of one cell's incoming values v;
// emit(I, value) receives post-collision population I::value, in increasing
// order.  Returns the cell's macroscopic values.
// Macroscopic values of one cell's incoming values v (the sums in velocity
// order, in P::Acc).
template <class M, class P>
__device__ __forceinline__ Macro cell_macro(const KParams& k, const typename P::S (&v)[M::Q]) {
    using A = typename P::Acc;
    A m0 = A(0), jx = A(0), jy = A(0), jz = A(0), en = A(0);
    static_for<M::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = M::table.e[i][0], ey = M::table.e[i][1], ez = M::table.e[i][2];
        constexpr int ee = M::table.e2[M::table.group[i]];
        const A vi = A(v[i]);
        m0 += vi;
        if constexpr (ex != 0) jx = fma(A(ex), vi, jx);
        if constexpr (ey != 0) jy = fma(A(ey), vi, jy);
        if constexpr (ez != 0) jz = fma(A(ez), vi, jz);
        if constexpr (ee != 0) en = fma(A(ee), vi, en);
    });
    return macro_from_sums<M::D, P::shifted>(k, m0, jx, jy, jz, en);
}

// cell_macro with its results pinned in registers: an empty asm statement
// that "modifies" them ends the compiler's view of how they were computed.
// Every update kernel takes its macroscopic values through this, so that the
// arithmetic after it (and the contraction of its multiply-adds into fused
// ones) is the same in the two-buffer and the in-place kernels and their
// results agree bit for bit.  It also keeps the in-place kernels, whose
// stores are predicated on active lanes, from moving the moment sums under
// that branch, where they were computed one sum after another with every
// converted value held live (register spills).
template <class M, class P>
__device__ __forceinline__ Macro cell_macro_pinned(const KParams& k,
                                                   const typename P::S (&v)[M::Q]) {
    Macro mc = cell_macro<M, P>(k, v);
    asm volatile("" : "+v"(mc.rho), "+v"(mc.dr), "+v"(mc.ux), "+v"(mc.uy), "+v"(mc.uz),
                 "+v"(mc.d), "+v"(mc.u2));
    return mc;
}

template <class M, class P, class Emit>
__device__ __forceinline__ void relax_with(const KParams& k, const typename P::S (&v)[M::Q],
                                           const Macro& mc, Emit&& emit);

template <class M, class P, class Emit>
__device__ __forceinline__ Macro relax_cell(const KParams& k, const typename P::S (&v)[M::Q],
                                            Emit&& emit) {
    const Macro mc = cell_macro_pinned<M, P>(k, v);
    relax_with<M, P>(k, v, mc, emit);
    return mc;
}

template <class M, class P, class Emit>
__device__ __forceinline__ void relax_with(const KParams& k, const typename P::S (&v)[M::Q],
                                           const Macro& mc, Emit&& emit) {
    using R = typename P::S;
    constexpr int G = M::G;
    constexpr int D = M::D;
    const R utx = R(mc.ux * k.invT0), uty = R(mc.uy * k.invT0), utz = R(mc.uz * k.invT0);
    const double wr = k.omega_eff * mc.rho;
    const double wd = k.omega_eff * mc.dr;
    const R omc = R(k.omc);
    const XPoly<D, M::N> xp(mc.u2, mc.d);

    static_for<G>([&](auto GI) {
        constexpr int g = decltype(GI)::value;
        const GCoef gc = xp.at(group_x<M, g>(k));
        const R a0 = R(gc.a0), a1 = R(gc.a1), a2 = R(gc.a2);
        const R ca = R(wr * k.W[g]);
        const R cb = R(wd * k.W[g]);
        static_for<M::table.gsize[g]>([&](auto JI) {
            constexpr int i = M::table.gstart[g] + decltype(JI)::value;
            constexpr int ex = M::table.e[i][0], ey = M::table.e[i][1], ez = M::table.e[i][2];
            const R s = edot<ex, ey, ez>(utx, uty, utz);
            const R h = horner_h<M::N>(a0, a1, a2, s);
            R out;
            if constexpr (P::shifted) {
                out = fma(omc, v[i], fma(ca, h, cb));
            } else {
                out = fma(ca, h, fma(omc, v[i], ca));
            }
            emit(std::integral_constant<int, i>{}, out);
        });
    });
}

// Forward update, two buffers: pull gather from src, relax, store to dst.
// STORE_MOM additionally writes the D+2 moments of the input state
// (delta rho or rho, U, theta - 1) for the adjoint.
//
// Relaxation: out = omc v + omega_eff W (dr + rho h)   (F32S)
//             out = omc v + omega_eff W rho (1 + h)    (F64)
// with omc + omega_eff = 1 exactly, so mass, momentum and energy are
// conserved up to the rounding of each cell's own values.
//
// HOLD: rows inside the held planes of the slowest axis (the fixed end
// planes of the shock tube) store f^eq of the held state instead; the test
// is uniform over a block.
// The stored step moments of a cell on a held plane: those of the held state.
template <class M, class P>
__device__ __forceinline__ void store_held_moments(const KParams& k, const Cell& cl,
                                                   const FixedState& st,
                                                   typename P::S* __restrict__ mom) {
    using S = typename P::S;
    if (!cl.active) return;
    mom[cl.c] = S(P::shifted ? st.rho - k.rho0 : st.rho);
    mom[k.N + cl.c] = S(st.U[0]);
    mom[2 * k.N + cl.c] = S(st.U[1]);
    if constexpr (M::D == 3) mom[3 * k.N + cl.c] = S(st.U[2]);
    mom[(M::D + 1) * k.N + cl.c] = S(st.T * k.invT0 - 1.0);
}

// POP = false (with STORE_MOM): the step's moments only, no populations are
// relaxed or stored (the last recomputed step of a checkpoint segment,
// whose post-collision state the next snapshot already holds).
template <class M, class P, bool STORE_MOM, bool HOLD, bool POP = true>
__global__ __launch_bounds__(row_block_limit(M::Q, P::id)) __attribute__((amdgpu_waves_per_eu(P::waves)))
void k_step(const typename P::S* __restrict__ src, typename P::S* __restrict__ dst, KParams k,
            typename P::S* __restrict__ mom) {
    using S = typename P::S;
    constexpr int D = M::D;
    static_assert(POP || STORE_MOM, "a step stores populations, moments or both");
    const Cell cl = row_cell<true>(k);

    if constexpr (HOLD) {
        const int sl = (D == 3) ? cl.z : cl.y;
        const int L = (D == 3) ? k.nz : k.ny;
        if (sl < k.hold_lo || sl >= L - k.hold_hi) {
            const FixedState& st = (sl < k.hold_lo) ? k.hold[0] : k.hold[1];
            if constexpr (POP) {
                PlaneWriter<S> out_w(dst, k, cl, M::Q);
                feq_cell<M, P>(k, st.rho, st.U[0], st.U[1], st.U[2], st.T,
                               [&](auto, S val) { out_w.put(val); });
            }
            if constexpr (STORE_MOM) store_held_moments<M, P>(k, cl, st, mom);
            return;
        }
    }

    S v[M::Q];
    gather<M, +1>(src, k, cl, v);
    Macro mc;
    if constexpr (POP) {
        PlaneWriter<S> out_w(dst, k, cl, M::Q);
        mc = relax_cell<M, P>(k, v, [&](auto, S val) { out_w.put(val); });
    } else {
        mc = cell_macro_pinned<M, P>(k, v);
    }

    if constexpr (STORE_MOM) {
        if (cl.active) {
            mom[cl.c] = S(P::shifted ? mc.dr : mc.rho);
            mom[k.N + cl.c] = S(mc.ux);
            mom[2 * k.N + cl.c] = S(mc.uy);
            if constexpr (D == 3) mom[3 * k.N + cl.c] = S(mc.uz);
            mom[(D + 1) * k.N + cl.c] = S(mc.d);
        }
    }
}

// Forward update in place on one buffer (AA pattern).  The buffer holds the
// post-collision state f* of the current step in one of two forms:
//   swapped : f*_i(x) in run opp(i) of cell x,
//   pushed  : f*_i(x) in run i of cell x + e_i (already streamed).
// PUSH = true  reads the swapped form: the value arriving at x along e_i is
//              run opp(i) of cell x - e_i; it relaxes and writes f*_i(x) to
//              run i of cell x + e_i (pushed form).
// PUSH = false reads the pushed form: run i of cell x is the arriving value;
//              it relaxes and writes f*_i(x) to run opp(i) of cell x
//              (swapped form).
// Every location is read and then written by the same thread only, so the
// update is race-free in place.  Idle lanes of a ragged row do not store
// (a duplicate store could overwrite a value before its reader loads it).
// HOLD: cells on the held end planes store f^eq of the held state into the
// same locations instead of reading them (as k_step<HOLD> does for the
// two-buffer step), so both schemes hold the same values.
// STORE_MOM: also store the step's D+2 moments, as k_step<STORE_MOM> does.
template <class M, class P, bool PUSH, bool HOLD, bool STORE_MOM>
__global__ __launch_bounds__(row_block_limit(M::Q, P::id)) __attribute__((amdgpu_waves_per_eu(P::waves)))
void k_step_aa(typename P::S* f, KParams k, typename P::S* __restrict__ mom) {
    using S = typename P::S;
    constexpr int D = M::D;
    const Cell cl = row_cell<true>(k);
    const SlabAddr<M, S, char> ad(reinterpret_cast<char*>(f), k, cl);
    const auto put = [&](auto I, S val) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = M::table.e[i][0], ey = M::table.e[i][1], ez = M::table.e[i][2];
        if (cl.active) {
            if constexpr (PUSH)
                store_pop<S, LBM_AA_NT_PUSH != 0>(ad.template at<i, ex, ey, ez>(), val);
            else
                store_pop<S, LBM_AA_NT_LOCAL != 0>(ad.template at<M::table.opp[i], 0, 0, 0>(), val);
        }
    };
    if constexpr (HOLD) {
        const int sl = (D == 3) ? cl.z : cl.y;
        const int L = (D == 3) ? k.nz : k.ny;
        if (sl < k.hold_lo || sl >= L - k.hold_hi) {
            const FixedState& st = (sl < k.hold_lo) ? k.hold[0] : k.hold[1];
            feq_cell<M, P>(k, st.rho, st.U[0], st.U[1], st.U[2], st.T, put);
            if constexpr (STORE_MOM) store_held_moments<M, P>(k, cl, st, mom);
            return;
        }
    }
    S v[M::Q];
    static_for<M::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = M::table.e[i][0], ey = M::table.e[i][1], ez = M::table.e[i][2];
        if constexpr (PUSH)
            v[i] = load_pop<S>(ad.template at<M::table.opp[i], -ex, -ey, -ez>());
        else
            v[i] = load_pop<S>(ad.template at<i, 0, 0, 0>());
    });
    const Macro mc = cell_macro_pinned<M, P>(k, v);
    relax_with<M, P>(k, v, mc, put);
    if constexpr (STORE_MOM) {
        if (cl.active) {
            mom[cl.c] = S(P::shifted ? mc.dr : mc.rho);
            mom[k.N + cl.c] = S(mc.ux);
            mom[2 * k.N + cl.c] = S(mc.uy);
            if constexpr (D == 3) mom[3 * k.N + cl.c] = S(mc.uz);
            mom[(D + 1) * k.N + cl.c] = S(mc.d);
        }
    }
}

// ---------------------------------------------------------------------------
// f = f^eq(rho, U, T) from float64 fields.
template <class M, class P, int FORM>
__global__ __launch_bounds__(kBlock) void k_init(const double* __restrict__ rho,
                                                 const double* __restrict__ U,
                                                 const double* __restrict__ T,
                                                 typename P::S* __restrict__ f, KParams k) {
    const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= k.N) return;
    store_feq<M, P, FORM>(f, k, c, rho[c], U[c], U[k.N + c], (M::D == 3) ? U[2 * k.N + c] : 0.0,
                          T[c]);
}

// Copy float64 f[Q][N] into storage, and back.
template <class M, class P, int FORM>
__global__ __launch_bounds__(kBlock) void k_set_pop(const double* __restrict__ fin,
                                                    typename P::S* __restrict__ f, KParams k) {
    const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= k.N) return;
    const PopAt<M, FORM> pa(k, c);
    static_for<M::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int g = M::table.group[i];
        const double val = fin[static_cast<long long>(i) * k.N + c];
        if constexpr (P::shifted)
            f[pa.template at<i>()] = static_cast<float>(val - k.W[g] * k.rho0);
        else
            f[pa.template at<i>()] = val;
    });
}

template <class M, class P, int FORM>
__global__ __launch_bounds__(kBlock) void k_get_pop(const typename P::S* __restrict__ f,
                                                    double* __restrict__ fout, KParams k) {
    const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= k.N) return;
    const PopAt<M, FORM> pa(k, c);
    static_for<M::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int g = M::table.group[i];
        const double val = static_cast<double>(f[pa.template at<i>()]);
        fout[static_cast<long long>(i) * k.N + c] = P::shifted ? val + k.W[g] * k.rho0 : val;
    });
}

// Copy of a stored state in form FORM into the two-buffer form (same
// storage type, bit for bit).
template <class M, class P, int FORM>
__global__ __launch_bounds__(kBlock) void k_to_ab(const typename P::S* __restrict__ f,
                                                  typename P::S* __restrict__ out, KParams k) {
    const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= k.N) return;
    const PopAt<M, FORM> src(k, c);
    const PopAt<M, kFormAB> dst(k, c);
    static_for<M::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        out[dst.template at<i>()] = f[src.template at<i>()];
    });
}

// The reverse: a state in the two-buffer form copied into form FORM.
template <class M, class P, int FORM>
__global__ __launch_bounds__(kBlock) void k_from_ab(const typename P::S* __restrict__ f,
                                                    typename P::S* __restrict__ out, KParams k) {
    const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= k.N) return;
    const PopAt<M, kFormAB> src(k, c);
    const PopAt<M, FORM> dst(k, c);
    static_for<M::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        out[dst.template at<i>()] = f[src.template at<i>()];
    });
}

// Raw float64 sums of one cell: sum v, sum v e, sum v |e|^2 of the stored values.
template <class M, int FORM, class S>
__device__ __forceinline__ void cell_sums(const S* __restrict__ f, const KParams& k, long long c,
                                          double& m0, double (&j)[3], double& en) {
    m0 = 0.0;
    j[0] = j[1] = j[2] = 0.0;
    en = 0.0;
    const PopAt<M, FORM> pa(k, c);
    static_for<M::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = M::table.e[i][0], ey = M::table.e[i][1], ez = M::table.e[i][2];
        constexpr int ee = M::table.e2[M::table.group[i]];
        const double val = static_cast<double>(f[pa.template at<i>()]);
        m0 += val;
        if constexpr (ex != 0) j[0] += double(ex) * val;
        if constexpr (ey != 0) j[1] += double(ey) * val;
        if constexpr (ez != 0) j[2] += double(ez) * val;
        if constexpr (ee != 0) en += double(ee) * val;
    });
}

template <class M, class P, int FORM>
__global__ __launch_bounds__(kBlock) void k_moments(const typename P::S* __restrict__ f,
                                                    double* __restrict__ rho, double* __restrict__ U,
                                                    double* __restrict__ T, KParams k) {
    constexpr int D = M::D;
    const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= k.N) return;
    double m0, j[3], en;
    cell_sums<M, FORM>(f, k, c, m0, j, en);
    double r, d;
    double u[3];
    if constexpr (P::shifted) {
        r = k.rho0 + m0;
        for (int a = 0; a < 3; ++a) u[a] = j[a] / r;
        const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        d = (en - D * k.T0 * m0 - r * usq) / (r * D * k.T0);
    } else {
        r = m0;
        for (int a = 0; a < 3; ++a) u[a] = j[a] / r;
        const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        d = (en / r - usq) / (D * k.T0) - 1.0;
    }
    if (rho) rho[c] = r;
    if (U) {
        for (int a = 0; a < D; ++a) U[a * k.N + c] = u[a];
    }
    if (T) T[c] = k.T0 * (1.0 + d);
}

// Conservation sums of the stored values, grid-stride, fixed order.
template <class M, class P, int FORM>
__global__ __launch_bounds__(kBlock) void k_conservation(const typename P::S* __restrict__ f,
                                                         KParams k, double* __restrict__ partials) {
    constexpr int D = M::D;
    double acc[D + 2];
    static_for<D + 2>([&](auto QI) { acc[decltype(QI)::value] = 0.0; });
    const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < k.N;
         c += stride) {
        double m0, j[3], en;
        cell_sums<M, FORM>(f, k, c, m0, j, en);
        acc[0] += m0;
        for (int a = 0; a < D; ++a) acc[1 + a] += j[a];
        acc[D + 1] += 0.5 * en;
    }
    block_sum<D + 2>(acc, partials + static_cast<long long>(blockIdx.x) * (D + 2), false);
}

// ---------------------------------------------------------------------------
// Adjoint.
//
// lambda^n_i(x) = dL/drho_n(x) for every i; partK[block] = sum dL/drho_n * rho_n.
// On held planes rho_n is the held state's, a constant: lambda^n = 0 there.
template <class M, class P>
__global__ __launch_bounds__(kBlock) void k_lambda_init(const typename P::S* __restrict__ fn,
                                                        const double* __restrict__ dLdrho,
                                                        typename P::S* __restrict__ lam,
                                                        KParams k, double* __restrict__ partK) {
    using S = typename P::S;
    const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    double acc[1] = {0.0};
    if (c < k.N) {
        const long long plane = static_cast<long long>(k.nx) * (M::D == 3 ? k.ny : 1);
        const long long sl = c / plane;
        const long long L = (M::D == 3) ? k.nz : k.ny;
        const bool held = sl < k.hold_lo || sl >= L - k.hold_hi;
        const double g = held ? 0.0 : dLdrho[c];
        double m0 = 0.0;
        const PopAt<M, kFormAB> pa(k, c);
        static_for<M::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            m0 += static_cast<double>(fn[pa.template at<i>()]);
            lam[pa.template at<i>()] = static_cast<S>(g);
        });
        const double r = P::shifted ? k.rho0 + m0 : m0;
        acc[0] = g * r;
    }
    block_sum<1>(acc, partK + blockIdx.x, false);
}

// Coefficients of h and of its derivatives with respect to s, u2 and d for
// one group, straight from (u2, d, X) (the adjoint kernels: per-cell
// polynomials in X, as the forward kernels use, would hold a dozen more
// float64 values through their group loop and push them past 3 waves per
// SIMD).  With K1 = (X - D)/2, K2 = (D + 2 - X)/4,
// K3 = (X^2 - 2(D + 2)X + D(D + 2))/8 (the file header's a0, a1, a2) and
//   N = 4: P_s  = a1 + s (2 a2 + s (1/2 + s/6))
//          P_u2 = b0 + s (-1/2 - s/4),   b0 = -1/2 + u2/4 + d K2
//          P_d  = c0 + s (c1 + s c2),     c0 = K1 + u2 K2 + 2 d K3,
//                                         c1 = (X - D - 2)/2, c2 = (X - D - 4)/4
//   N = 2: P_s = 1 + s, P_u2 = -1/2, P_d = (X - D)/2.
struct GDer {
    double b0, c0, c1, c2;
};
template <int D, int N>
__device__ __forceinline__ void group_coef_der(double u2, double d, double X, GCoef& gc,
                                               GDer& gd) {
    constexpr double Dd = D;
    if constexpr (N == 4) {
        const double k1 = 0.5 * (X - Dd), k2 = 0.25 * (Dd + 2.0 - X);
        const double k3 = 0.125 * (X * X - 2.0 * (Dd + 2.0) * X + Dd * (Dd + 2.0));
        gc.a0 = -0.5 * u2 + 0.125 * u2 * u2 + d * (k1 + u2 * k2 + d * k3);
        gc.a1 = 1.0 - 0.5 * u2 + d * (0.5 * (X - Dd - 2.0));
        gc.a2 = 0.5 - 0.25 * u2 + d * (0.25 * (X - Dd - 4.0));
        gd.b0 = -0.5 + 0.25 * u2 + d * k2;
        gd.c0 = k1 + u2 * k2 + 2.0 * d * k3;
        gd.c1 = 0.5 * (X - Dd - 2.0);
        gd.c2 = 0.25 * (X - Dd - 4.0);
    } else {
        static_assert(N == 2, "equilibrium order 2 or 4");
        gc.a0 = 0.5 * (-u2 + d * (X - Dd));
        gc.a1 = 1.0;
        gc.a2 = 0.5;
        gd.b0 = -0.5;
        gd.c0 = 0.5 * (X - Dd);
        gd.c1 = 0.0;
        gd.c2 = 0.0;
    }
}

// P_s, P_u2, P_d of order N from the group's coefficients.
template <int N, class R>
__device__ __forceinline__ R eq_ps(R a1, R a2x2, R s) {
    if constexpr (N == 4) return fma(s, fma(s, fma(s, R(1.0 / 6.0), R(0.5)), a2x2), a1);
    else return R(1) + s;
}
template <int N, class R>
__device__ __forceinline__ R eq_pu(R b0, R s) {
    if constexpr (N == 4) return fma(s, fma(s, R(-0.25), R(-0.5)), b0);
    else return R(-0.5);
}
template <int N, class R>
__device__ __forceinline__ R eq_pd(R c0, R c1, R c2, R s) {
    if constexpr (N == 4) return fma(s, fma(s, c2, c1), c0);
    else return c0;
}

// One transposed step.  mu_i = lambda^{t+1}_i(x + e_i); the moments of f^t at x
// come from the recomputation.  With f^eq_i = w_i rho P_i(U, T):
//   S0 = sum mu w P, Su = sum mu w P_u2, Sd = sum mu w P_d, Ss = sum mu w P_s e
//   dA/dU = rho/T0 (Ss + 2 U Su), dA/dT = rho/T0 Sd     (A = sum mu f^eq)
// and the chain rule to m = (rho, j = rho U, E = sum f |e|^2) gives
//   G_rho = S0 - dA/dU . U / rho + dA/dT (|U|^2 - D T) / (D rho)
//   G_j   = dA/dU / rho - 2 dA/dT U / (D rho),   G_E = dA/dT / (D rho).
// Output lambda^t_i = omc mu_i + omega (G_rho + G_j . e_i + G_E |e_i|^2).
// partA[block] += sum over the block's cells of A = rho S0.
// MARK: also partM[block] = sum over the block's cells of sum_i mu_i B_i with
// B the stored state the forward run streamed into f^{t+1} (a checkpoint),
// i.e. the invariant <lambda^{t+1}, f^{t+1}> of the step's homogeneity.
// The MARK instances (one step per checkpoint segment) hold the mark's loads
// as well and may use up to 256 registers (2 waves per SIMD instead of 3) to
// avoid spilling.
// HOLD: the post-collision values of cells on held planes are constants, so
// their adjoint state is zero (the cells are computed like the others and
// their output replaced, keeping every wave on the same barriers).
template <class M, class P, bool COLLIDE, bool MARK, bool HOLD>
__global__ __launch_bounds__(row_block_limit(M::Q, P::id))
__attribute__((amdgpu_waves_per_eu(MARK ? (P::adj_waves < 2 ? P::adj_waves : 2) : P::adj_waves)))
void k_adjoint(const typename P::S* __restrict__ lsrc, typename P::S* __restrict__ ldst,
               const typename P::S* __restrict__ mom, KParams k, double* __restrict__ partA,
               const typename P::S* __restrict__ mark_state, double* __restrict__ partM) {
    using S = typename P::S;
    using R = S;
    constexpr int Q = M::Q;
    constexpr int G = M::G;
    constexpr int D = M::D;
    const Cell cl = row_cell(k);

    S mu[Q];
    gather<M, -1>(lsrc, k, cl, mu);

    // MARK: mu_i B_i is accumulated where mu_i is consumed (the output loop
    // of the transposed streaming, the group sums of the collision), so
    // that the mark's loads do not extend the lifetime of mu.
    const SlabAddr<M, S, const char> mark_at(reinterpret_cast<const char*>(mark_state), k, cl);
    double mk = 0.0;
    const auto mark_term = [&](auto I) {
        if constexpr (MARK) {
            constexpr int i = decltype(I)::value;
            double b = static_cast<double>(load_pop<S>(mark_at.template at<i, 0, 0, 0>()));
            if constexpr (P::shifted) b += k.W[M::table.group[i]] * k.rho0;
            mk = fma(static_cast<double>(mu[i]), b, mk);
        }
    };

    if constexpr (!COLLIDE) {
        // transposed streaming only
        PlaneWriter<S> wt(ldst, k, cl, Q);
        static_for<Q>([&](auto I) {
            mark_term(I);
            wt.put(mu[decltype(I)::value]);
        });
        if constexpr (MARK) {
            double acc[1] = {cl.active ? mk : 0.0};
            block_sum<1>(acc, partM + blockIdx.x, false);
        }
        return;
    }

    const double m0 = static_cast<double>(mom[cl.c]);
    const double ux = static_cast<double>(mom[k.N + cl.c]);
    const double uy = static_cast<double>(mom[2 * k.N + cl.c]);
    const double uz = (D == 3) ? static_cast<double>(mom[3 * k.N + cl.c]) : 0.0;
    const double d = static_cast<double>(mom[(D + 1) * k.N + cl.c]);
    const double rho = P::shifted ? k.rho0 + m0 : m0;
    const double usq = ux * ux + uy * uy + uz * uz;
    const double u2 = usq * k.invT0;
    const R utx = R(ux * k.invT0), uty = R(uy * k.invT0), utz = R(uz * k.invT0);

    // Group sums in storage precision, combined with the float64 weights in
    // float64: rounding the weights would make this the transpose of a
    // slightly different model than the forward step and bias the omega
    // gradient, which relies on <lambda^t, f*^t> staying constant.
    double s0 = 0.0, su2 = 0.0, sd = 0.0, ssx = 0.0, ssy = 0.0, ssz = 0.0;
    static_for<G>([&](auto GI) {
        constexpr int g = decltype(GI)::value;
        GCoef gc;
        GDer gd;
        group_coef_der<D, M::N>(u2, d, group_x<M, g>(k), gc, gd);
        const R a0 = R(gc.a0), a1 = R(gc.a1), a2 = R(gc.a2), a2x2 = R(2.0 * gc.a2);
        const R b0 = R(gd.b0), c0 = R(gd.c0), c1 = R(gd.c1), c2 = R(gd.c2);
        // sum mu P = sum mu + sum mu h with P = 1 + h: the O(1) part is summed in
        // float64 so that the small omega signal in A is not lost to rounding.
        double tm = 0.0;
        R t0 = R(0), tu = R(0), td = R(0), tx = R(0), ty = R(0), tz = R(0), tb = R(0);
        static_for<M::table.gsize[g]>([&](auto JI) {
            constexpr int i = M::table.gstart[g] + decltype(JI)::value;
            constexpr int ex = M::table.e[i][0], ey = M::table.e[i][1], ez = M::table.e[i][2];
            const R s = edot<ex, ey, ez>(utx, uty, utz);
            const R h = horner_h<M::N>(a0, a1, a2, s);
            const R ps = eq_ps<M::N>(a1, a2x2, s);
            const R pu = eq_pu<M::N>(b0, s);
            const R pd = eq_pd<M::N>(c0, c1, c2, s);
            tm += static_cast<double>(mu[i]);
            if constexpr (MARK) tb = fma(mu[i], load_pop<S>(mark_at.template at<i, 0, 0, 0>()), tb);
            t0 = fma(mu[i], h, t0);
            tu = fma(mu[i], pu, tu);
            td = fma(mu[i], pd, td);
            const R t = mu[i] * ps;
            if constexpr (ex != 0) tx = fma(R(ex), t, tx);
            if constexpr (ey != 0) ty = fma(R(ey), t, ty);
            if constexpr (ez != 0) tz = fma(R(ez), t, tz);
        });
        const double wg = k.W[g];
        if constexpr (MARK) {
            // sum_i mu_i B_i of the group: the stored part in storage precision,
            // the shift w_g rho0 sum_i mu_i from the float64 group sum
            mk += double(tb);
            if constexpr (P::shifted) mk = fma(wg * k.rho0, tm, mk);
        }
        s0 = fma(wg, tm + double(t0), s0);
        su2 = fma(wg, double(tu), su2);
        sd = fma(wg, double(td), sd);
        ssx = fma(wg, double(tx), ssx);
        ssy = fma(wg, double(ty), ssy);
        ssz = fma(wg, double(tz), ssz);
    });

    // chain rule in float64
    const double rT = rho * k.invT0;
    const double aux = rT * (ssx + 2.0 * ux * su2);
    const double auy = rT * (ssy + 2.0 * uy * su2);
    const double auz = rT * (ssz + 2.0 * uz * su2);
    const double at = rT * sd;
    const double invr = 1.0 / rho;
    const double Tm = k.T0 * (1.0 + d);
    const double grho = s0 - invr * (aux * ux + auy * uy + auz * uz) +
                        at * (usq - D * Tm) * invr * (1.0 / D);
    const double k2 = (2.0 / D) * at * invr;
    const double w = k.omega_eff;
    const R gjx = R(w * (aux * invr - k2 * ux));
    const R gjy = R(w * (auy * invr - k2 * uy));
    const R gjz = R(w * (auz * invr - k2 * uz));
    const R ge = R(w * at * invr * (1.0 / D));
    const R gr = R(w * grho);
    const R omc = R(k.omc);
    PlaneWriter<S> out_w(ldst, k, cl, Q);
    bool held = false;
    if constexpr (HOLD) {
        const int sl = (D == 3) ? cl.z : cl.y;
        const int L = (D == 3) ? k.nz : k.ny;
        held = sl < k.hold_lo || sl >= L - k.hold_hi;
    }

    static_for<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = M::table.e[i][0], ey = M::table.e[i][1], ez = M::table.e[i][2];
        constexpr int ee = M::table.e2[M::table.group[i]];
        R hv = gr;
        if constexpr (ee != 0) hv = fma(R(ee), ge, hv);
        if constexpr (ex != 0) hv = fma(R(ex), gjx, hv);
        if constexpr (ey != 0) hv = fma(R(ey), gjy, hv);
        if constexpr (ez != 0) hv = fma(R(ez), gjz, hv);
        const S out = fma(omc, mu[i], hv);
        if constexpr (HOLD) out_w.put(held ? S(0) : out);
        else out_w.put(out);
    });

    if constexpr (MARK) {
        double acc[2] = {cl.active ? rho * s0 : 0.0, cl.active ? mk : 0.0};
        block_sum_with<2>(acc, [&](int q, double v) {
            if (q == 0) partA[blockIdx.x] += v;
            else partM[blockIdx.x] = v;
        });
    } else {
        double acc[1] = {(cl.active && !held) ? rho * s0 : 0.0};
        block_sum<1>(acc, partA + blockIdx.x, true);
    }
}

// dL/dT_init(x) = sum_i lambda^0_i(x) d f_i^eq / dT at the initial fields,
// = rho / T0 sum_i lambda_i w_i P_d,i.
template <class M, class P>
__global__ __launch_bounds__(kBlock) void k_dT_init(const typename P::S* __restrict__ lam,
                                                    const double* __restrict__ rho,
                                                    const double* __restrict__ U,
                                                    const double* __restrict__ T,
                                                    double* __restrict__ dT, KParams k) {
    constexpr int D = M::D;
    constexpr int G = M::G;
    const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= k.N) return;
    const double r = rho[c];
    const double ux = U[c], uy = U[k.N + c], uz = (D == 3) ? U[2 * k.N + c] : 0.0;
    const double d = T[c] * k.invT0 - 1.0;
    const double u2 = (ux * ux + uy * uy + uz * uz) * k.invT0;
    const double utx = ux * k.invT0, uty = uy * k.invT0, utz = uz * k.invT0;
    const PopAt<M, kFormAB> pa(k, c);
    double sd = 0.0;
    static_for<G>([&](auto GI) {
        constexpr int g = decltype(GI)::value;
        GCoef gc;
        GDer gd;
        group_coef_der<D, M::N>(u2, d, group_x<M, g>(k), gc, gd);
        double tg = 0.0;
        static_for<M::table.gsize[g]>([&](auto JI) {
            constexpr int i = M::table.gstart[g] + decltype(JI)::value;
            constexpr int ex = M::table.e[i][0], ey = M::table.e[i][1], ez = M::table.e[i][2];
            const double s = edot<ex, ey, ez>(utx, uty, utz);
            const double pd = eq_pd<M::N>(gd.c0, gd.c1, gd.c2, s);
            tg += static_cast<double>(lam[pa.template at<i>()]) * pd;
        });
        sd += k.W[g] * tg;
    });
    dT[c] = r * k.invT0 * sd;
}

inline unsigned cell_blocks(long long N) {
    return static_cast<unsigned>((N + kBlock - 1) / kBlock);
}

static_assert(kBlock == kReduceThreads, "reduce_blocks (host) assumes kBlock threads");

// Calls f with std::integral_constant<int, kp.form>.
template <class F>
hipError_t with_form(const KParams& kp, F&& f) {
    if (kp.form == kFormPushed) return f(std::integral_constant<int, kFormPushed>{});
    if (kp.form == kFormSwapped) return f(std::integral_constant<int, kFormSwapped>{});
    return f(std::integral_constant<int, kFormAB>{});
}

// Same for the forms a kernel that writes a whole state starts from.
template <class F>
hipError_t with_initial_form(const KParams& kp, F&& f) {
    if (kp.form == kFormSwapped) return f(std::integral_constant<int, kFormSwapped>{});
    return f(std::integral_constant<int, kFormAB>{});
}

}  // namespace

template <class M, Prec PR>
hipError_t ModelKernels<M, PR>::init(const KParams& kp, const double* rho, const double* U,
                                     const double* T, void* f, hipStream_t s) {
    using P = typename PrecOf<PR>::type;
    return with_initial_form(kp, [&](auto F) {
        hipLaunchKernelGGL((k_init<M, P, decltype(F)::value>), dim3(cell_blocks(kp.N)),
                           dim3(kBlock), 0, s, rho, U, T, static_cast<typename P::S*>(f), kp);
        return hipGetLastError();
    });
}

template <class M, Prec PR>
hipError_t ModelKernels<M, PR>::set_pop(const KParams& kp, const double* fin, void* f,
                                        hipStream_t s) {
    using P = typename PrecOf<PR>::type;
    return with_initial_form(kp, [&](auto F) {
        hipLaunchKernelGGL((k_set_pop<M, P, decltype(F)::value>), dim3(cell_blocks(kp.N)),
                           dim3(kBlock), 0, s, fin, static_cast<typename P::S*>(f), kp);
        return hipGetLastError();
    });
}

template <class M, Prec PR>
hipError_t ModelKernels<M, PR>::get_pop(const KParams& kp, const void* f, double* fout,
                                        hipStream_t s) {
    using P = typename PrecOf<PR>::type;
    return with_form(kp, [&](auto F) {
        hipLaunchKernelGGL((k_get_pop<M, P, decltype(F)::value>), dim3(cell_blocks(kp.N)),
                           dim3(kBlock), 0, s, static_cast<const typename P::S*>(f), fout, kp);
        return hipGetLastError();
    });
}

template <class M, Prec PR>
hipError_t ModelKernels<M, PR>::step(const KParams& kp, const void* src, void* dst,
                                     void* mom_out, hipStream_t s) {
    using P = typename PrecOf<PR>::type;
    using S = typename P::S;
    const dim3 grid(static_cast<unsigned>(step_blocks(M::id, PR, kp)));
    const auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, grid, dim3(kp.bx), 0, s,
                           static_cast<const S*>(src), static_cast<S*>(dst), kp,
                           static_cast<S*>(mom_out));
    };
    const bool hold = kp.hold_lo + kp.hold_hi > 0;
    if (mom_out && !dst) {
        if (hold) go(k_step<M, P, true, true, false>);
        else go(k_step<M, P, true, false, false>);
    } else if (mom_out) {
        if (hold) go(k_step<M, P, true, true>);
        else go(k_step<M, P, true, false>);
    } else {
        if (hold) go(k_step<M, P, false, true>);
        else go(k_step<M, P, false, false>);
    }
    return hipGetLastError();
}

template <class M, Prec PR>
hipError_t ModelKernels<M, PR>::step_aa(const KParams& kp, void* f, bool push, void* mom_out,
                                        hipStream_t s) {
    using P = typename PrecOf<PR>::type;
    using S = typename P::S;
    const dim3 grid(static_cast<unsigned>(step_blocks(M::id, PR, kp)));
    const auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, grid, dim3(kp.bx), 0, s, static_cast<S*>(f), kp,
                           static_cast<S*>(mom_out));
    };
    const bool hold = kp.hold_lo + kp.hold_hi > 0;
    if (push) {
        if (mom_out && hold) go(k_step_aa<M, P, true, true, true>);
        else if (mom_out) go(k_step_aa<M, P, true, false, true>);
        else if (hold) go(k_step_aa<M, P, true, true, false>);
        else go(k_step_aa<M, P, true, false, false>);
    } else {
        if (mom_out && hold) go(k_step_aa<M, P, false, true, true>);
        else if (mom_out) go(k_step_aa<M, P, false, false, true>);
        else if (hold) go(k_step_aa<M, P, false, true, false>);
        else go(k_step_aa<M, P, false, false, false>);
    }
    return hipGetLastError();
}

template <class M, Prec PR>
hipError_t ModelKernels<M, PR>::to_ab(const KParams& kp, const void* f, void* out,
                                      hipStream_t s) {
    using P = typename PrecOf<PR>::type;
    using S = typename P::S;
    return with_form(kp, [&](auto F) {
        hipLaunchKernelGGL((k_to_ab<M, P, decltype(F)::value>), dim3(cell_blocks(kp.N)),
                           dim3(kBlock), 0, s, static_cast<const S*>(f), static_cast<S*>(out), kp);
        return hipGetLastError();
    });
}

template <class M, Prec PR>
hipError_t ModelKernels<M, PR>::from_ab(const KParams& kp, const void* f, void* out,
                                        hipStream_t s) {
    using P = typename PrecOf<PR>::type;
    using S = typename P::S;
    return with_initial_form(kp, [&](auto F) {
        hipLaunchKernelGGL((k_from_ab<M, P, decltype(F)::value>), dim3(cell_blocks(kp.N)),
                           dim3(kBlock), 0, s, static_cast<const S*>(f), static_cast<S*>(out), kp);
        return hipGetLastError();
    });
}

template <class M, Prec PR>
hipError_t ModelKernels<M, PR>::moments(const KParams& kp, const void* f, double* rho, double* U,
                                        double* T, hipStream_t s) {
    using P = typename PrecOf<PR>::type;
    return with_form(kp, [&](auto F) {
        hipLaunchKernelGGL((k_moments<M, P, decltype(F)::value>), dim3(cell_blocks(kp.N)),
                           dim3(kBlock), 0, s, static_cast<const typename P::S*>(f), rho, U, T, kp);
        return hipGetLastError();
    });
}

template <class M, Prec PR>
hipError_t ModelKernels<M, PR>::conservation(const KParams& kp, const void* f, double* partials,
                                             hipStream_t s) {
    using P = typename PrecOf<PR>::type;
    const int nb = reduce_blocks(kp.N);
    return with_form(kp, [&](auto F) {
        hipLaunchKernelGGL((k_conservation<M, P, decltype(F)::value>), dim3(nb), dim3(kBlock), 0,
                           s, static_cast<const typename P::S*>(f), kp, partials);
        return hipGetLastError();
    });
}

template <class M, Prec PR>
hipError_t ModelKernels<M, PR>::lambda_init(const KParams& kp, const void* fn,
                                            const double* dLdrho, void* lam, double* partK,
                                            hipStream_t s) {
    using P = typename PrecOf<PR>::type;
    using S = typename P::S;
    hipLaunchKernelGGL((k_lambda_init<M, P>), dim3(cell_blocks(kp.N)), dim3(kBlock), 0, s,
                       static_cast<const S*>(fn), dLdrho, static_cast<S*>(lam), kp, partK);
    return hipGetLastError();
}

template <class M, Prec PR>
hipError_t ModelKernels<M, PR>::adjoint_step(const KParams& kp, const void* lam_src,
                                             void* lam_dst, const void* mom, double* partA,
                                             const void* mark_state, double* partM,
                                             hipStream_t s) {
    using P = typename PrecOf<PR>::type;
    using S = typename P::S;
    const long long blocks = step_blocks(M::id, PR, kp);
    const auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(static_cast<unsigned>(blocks)), dim3(kp.bx), 0, s,
                           static_cast<const S*>(lam_src), static_cast<S*>(lam_dst),
                           static_cast<const S*>(mom), kp, partA,
                           static_cast<const S*>(mark_state), partM);
    };
    const bool hold = kp.hold_lo + kp.hold_hi > 0;
    if (mom) {
        // (the omega marks are not taken with held planes)
        if (hold) go(k_adjoint<M, P, true, false, true>);
        else if (mark_state) go(k_adjoint<M, P, true, true, false>);
        else go(k_adjoint<M, P, true, false, false>);
    } else {
        if (mark_state) go(k_adjoint<M, P, false, true, false>);
        else go(k_adjoint<M, P, false, false, false>);
    }
    return hipGetLastError();
}

template <class M, Prec PR>
hipError_t ModelKernels<M, PR>::dT_init(const KParams& kp, const void* lam0, const double* rho,
                                        const double* U, const double* T, double* dT,
                                        hipStream_t s) {
    using P = typename PrecOf<PR>::type;
    hipLaunchKernelGGL((k_dT_init<M, P>), dim3(cell_blocks(kp.N)), dim3(kBlock), 0, s,
                       static_cast<const typename P::S*>(lam0), rho, U, T, dT, kp);
    return hipGetLastError();
}

}  // namespace lbm
