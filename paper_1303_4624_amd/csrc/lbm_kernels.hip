// lbm_kernels.hip - HIP kernels for CDNA4 (gfx950) of the thermal lattice
// Boltzmann update with the D2Q33 / D3Q95 on-lattice models.
//
// Data layout: structure of arrays, population i of cell c at i*N + c, cells
// x-fastest.  One thread owns one cell.  Every population read is a contiguous
// run of a grid row (neighbouring threads read neighbouring x), so the
// gather f_i(x - e_i) is coalesced; the x-wrap of the periodic grid is folded
// into the per-lane index, the y/z-wrap into a wave-uniform row offset.
//
// Precision variants:
//   F64  : f_i stored and computed in float64.
//   F32S : g_i = f_i - w_i rho0 stored and computed in float32; the moments
//          are formed from g (delta rho, j, sum g|e|^2) and the relaxation is
//          written for g, so the O(1) part w_i rho0 never enters float32
//          arithmetic.
//
// Equilibrium: the 4th-order Hermite expansion of the Maxwellian, written as
// a polynomial in s = xi_i . u_hat for each symmetry group (|e_i|^2 is
// constant on a group, so every coefficient except s is per group):
//   P_i = 1 + h_i,  h_i = a0 + s (a1 + s (a2 + s (1/6 + s/24)))
//   a0 = (-u2 + d (X - D)) / 2
//        + (3 u2^2 + 6 d (D + 2 - X) u2 + 3 d^2 (X^2 - 2 (D + 2) X + D (D + 2))) / 24
//   a1 = 1 - u2/2 + d (X - D - 2)/2,   a2 = 1/2 - u2/4 + d (X - D - 4)/4
// with xi_i = e_i / c_s, c_s^2 = T0, u_hat = U / c_s, u2 = |u_hat|^2,
// X = |xi_i|^2 and d = T/T0 - 1.  This is the contraction of
// sum_{n<=4} a^(n):H^(n)(xi)/n! with the Hermite coefficients of the
// Maxwellian, collected in powers of s.
#include <hip/hip_runtime.h>

#include <utility>

#include "lbm_internal.h"

namespace lbm {
namespace {

constexpr int kBlock = 256;            // threads per block of every kernel
constexpr int kW = 2 * kMaxDisp + 1;   // distinct displacement components

template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(static_cast<F&&>(f), std::make_integer_sequence<int, N>{});
}

struct F64T {
    using S = double;
    static constexpr bool shifted = false;
};
struct F32ST {
    using S = float;
    static constexpr bool shifted = true;
};

template <class R>
__device__ __forceinline__ R kp_w(const KParams& k, int g) {
    if constexpr (sizeof(R) == 8) return k.W[g]; else return k.Wf[g];
}
template <class R>
__device__ __forceinline__ R kp_x(const KParams& k, int g) {
    if constexpr (sizeof(R) == 8) return k.X[g]; else return k.Xf[g];
}
template <class R>
__device__ __forceinline__ R kp_omega(const KParams& k) {
    if constexpr (sizeof(R) == 8) return k.omega; else return k.omegaf;
}
template <class R>
__device__ __forceinline__ R kp_T0(const KParams& k) {
    if constexpr (sizeof(R) == 8) return k.T0; else return k.T0f;
}
template <class R>
__device__ __forceinline__ R kp_invT0(const KParams& k) {
    if constexpr (sizeof(R) == 8) return 1.0 / k.T0; else return k.invT0f;
}
template <class R>
__device__ __forceinline__ R kp_rho0(const KParams& k) {
    if constexpr (sizeof(R) == 8) return k.rho0; else return k.rho0f;
}

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
    bool active;
    long long c;        // linear cell index
};

// Row-blocked mapping: block b covers threads [chunk*bx, chunk*bx + bx) of
// grid row `row` = y + ny*z.  y and z are uniform over the block.
__device__ __forceinline__ Cell row_cell(const KParams& k) {
    const int b = blockIdx.x;
    const int chunk = b % k.chunks;
    const int row = b / k.chunks;
    Cell cl;
    const int x = chunk * k.bx + static_cast<int>(threadIdx.x);
    cl.active = x < k.nx;
    cl.x = cl.active ? x : 0;
    cl.y = row % k.ny;
    cl.z = row / k.ny;
    cl.c = (static_cast<long long>(row)) * k.nx + cl.x;
    return cl;
}

// Gather v_i = src_i(x - SIGN*e_i) with periodic wrap on every axis.
// SIGN = +1 is the pull of the forward update, SIGN = -1 the transposed
// (adjoint) streaming.
template <class M, int SIGN, class S>
__device__ __forceinline__ void gather(const S* __restrict__ src, const KParams& k, const Cell& cl,
                                       S (&v)[M::Q]) {
    int xw[kW], yw[kW], zw[kW];
    static_for<kW>([&](auto DI) {
        constexpr int d = decltype(DI)::value - kMaxDisp;
        xw[d + kMaxDisp] = wrap_idx(cl.x - d, k.nx);
        yw[d + kMaxDisp] = wrap_idx(cl.y - d, k.ny);
        zw[d + kMaxDisp] = (M::D == 3) ? wrap_idx(cl.z - d, k.nz) : 0;
    });
    static_for<M::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = SIGN * M::table.e[i][0];
        constexpr int ey = SIGN * M::table.e[i][1];
        constexpr int ez = SIGN * M::table.e[i][2];
        const long long roff =
            (static_cast<long long>(zw[ez + kMaxDisp]) * k.ny + yw[ey + kMaxDisp]) * k.nx;
        const S* p = src + static_cast<long long>(i) * k.N + roff;
        v[i] = p[xw[ex + kMaxDisp]];
    });
}

// Per-group coefficients of h = P - 1 as a polynomial in s.
template <int D, class R>
struct Herm {
    R a0, a1, a2;   // h = a0 + s (a1 + s (a2 + s (1/6 + s/24)))
    __device__ __forceinline__ void set(R X, R u2, R d) {
        const R Dr = R(D);
        a0 = R(0.5) * (d * (X - Dr) - u2) +
             R(1.0 / 24.0) * (R(3) * u2 * u2 + R(6) * d * (Dr + R(2) - X) * u2 +
                              R(3) * d * d * (X * X - R(2) * (Dr + R(2)) * X + Dr * (Dr + R(2))));
        a1 = R(1) - R(0.5) * u2 + R(0.5) * d * (X - Dr - R(2));
        a2 = R(0.5) - R(0.25) * u2 + R(0.25) * d * (X - Dr - R(4));
    }
    __device__ __forceinline__ R h(R s) const {
        return a0 + s * (a1 + s * (a2 + s * (R(1.0 / 6.0) + s * R(1.0 / 24.0))));
    }
};

// s_i = e_i . ut with compile-time integer components.
template <int ex, int ey, int ez, class R>
__device__ __forceinline__ R edot(R ux, R uy, R uz) {
    R s = R(0);
    if constexpr (ex != 0) s = R(ex) * ux;
    if constexpr (ey != 0) s = (ex != 0) ? s + R(ey) * uy : R(ey) * uy;
    if constexpr (ez != 0) s = (ex != 0 || ey != 0) ? s + R(ez) * uz : R(ez) * uz;
    return s;
}

// Sum over a block of K doubles per thread; thread 0 writes (or adds to) out[0..K).
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* out, bool accumulate) {
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
            out[q] = accumulate ? out[q] + s : s;
        });
    }
}

// ---------------------------------------------------------------------------
// Forward update: pull gather, moments, equilibrium, BGK relaxation, store.
// STORE_MOM additionally writes the D+2 moments of the input state
// (delta rho or rho, U, theta - 1) for the adjoint.
template <class M, class P, bool STORE_MOM>
__global__ __launch_bounds__(kBlock) void k_step(const typename P::S* __restrict__ src,
                                                 typename P::S* __restrict__ dst, KParams k,
                                                 typename P::S* __restrict__ mom) {
    using S = typename P::S;
    using R = S;
    constexpr int Q = M::Q;
    constexpr int G = M::G;
    constexpr int D = M::D;
    const Cell cl = row_cell(k);

    S v[Q];
    gather<M, +1>(src, k, cl, v);

    R m0 = R(0), jx = R(0), jy = R(0), jz = R(0), en = R(0);
    static_for<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = M::table.e[i][0], ey = M::table.e[i][1], ez = M::table.e[i][2];
        constexpr int ee = M::table.e2[M::table.group[i]];
        m0 += v[i];
        if constexpr (ex != 0) jx += R(ex) * v[i];
        if constexpr (ey != 0) jy += R(ey) * v[i];
        if constexpr (ez != 0) jz += R(ez) * v[i];
        if constexpr (ee != 0) en += R(ee) * v[i];
    });

    const R T0 = kp_T0<R>(k);
    const R invT0 = kp_invT0<R>(k);
    const R omega = kp_omega<R>(k);
    const R omc = R(1) - omega;
    R rho, dr;
    if constexpr (P::shifted) {
        dr = m0;
        rho = kp_rho0<R>(k) + dr;
    } else {
        rho = m0;
        dr = R(0);
    }
    const R inv = R(1) / rho;
    const R ux = jx * inv, uy = jy * inv, uz = (D == 3) ? jz * inv : R(0);
    const R usq = ux * ux + uy * uy + uz * uz;
    const R invDT0 = invT0 * R(1.0 / D);
    R d;
    if constexpr (P::shifted) {
        d = (en - R(D) * T0 * dr - rho * usq) * inv * invDT0;
    } else {
        d = (en * inv - usq) * invDT0 - R(1);
    }
    const R utx = ux * invT0, uty = uy * invT0, utz = uz * invT0;
    const R u2 = usq * invT0;

    Herm<D, R> hc[G];
    R ca[G], cb[G];
    static_for<G>([&](auto GI) {
        constexpr int g = decltype(GI)::value;
        hc[g].set(kp_x<R>(k, g), u2, d);
        const R ow = omega * kp_w<R>(k, g);
        ca[g] = ow * rho;
        cb[g] = ow * dr;
    });

    static_for<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int g = M::table.group[i];
        constexpr int ex = M::table.e[i][0], ey = M::table.e[i][1], ez = M::table.e[i][2];
        const R s = edot<ex, ey, ez>(utx, uty, utz);
        const R h = hc[g].h(s);
        R out;
        if constexpr (P::shifted) {
            out = fma(omc, v[i], fma(ca[g], h, cb[g]));
        } else {
            out = fma(ca[g], h, fma(omc, v[i], ca[g]));
        }
        if (cl.active) dst[static_cast<long long>(i) * k.N + cl.c] = out;
    });

    if constexpr (STORE_MOM) {
        if (cl.active) {
            mom[cl.c] = P::shifted ? dr : rho;
            mom[k.N + cl.c] = ux;
            mom[2 * k.N + cl.c] = uy;
            if constexpr (D == 3) mom[3 * k.N + cl.c] = uz;
            mom[(D + 1) * k.N + cl.c] = d;
        }
    }
}

// ---------------------------------------------------------------------------
// f = f^eq(rho, U, T) from float64 fields, computed in float64.
template <class M, class P>
__global__ __launch_bounds__(kBlock) void k_init(const double* __restrict__ rho,
                                                 const double* __restrict__ U,
                                                 const double* __restrict__ T,
                                                 typename P::S* __restrict__ f, KParams k) {
    constexpr int D = M::D;
    constexpr int G = M::G;
    const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= k.N) return;
    const double r = rho[c];
    const double ux = U[c], uy = U[k.N + c], uz = (D == 3) ? U[2 * k.N + c] : 0.0;
    const double invT0 = 1.0 / k.T0;
    const double d = T[c] * invT0 - 1.0;
    const double u2 = (ux * ux + uy * uy + uz * uz) * invT0;
    const double utx = ux * invT0, uty = uy * invT0, utz = uz * invT0;
    Herm<D, double> hc[G];
    static_for<G>([&](auto GI) {
        constexpr int g = decltype(GI)::value;
        hc[g].set(k.X[g], u2, d);
    });
    static_for<M::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int g = M::table.group[i];
        constexpr int ex = M::table.e[i][0], ey = M::table.e[i][1], ez = M::table.e[i][2];
        const double h = hc[g].h(edot<ex, ey, ez>(utx, uty, utz));
        const double w = k.W[g];
        if constexpr (P::shifted) {
            f[static_cast<long long>(i) * k.N + c] =
                static_cast<float>(w * (r - k.rho0) + w * r * h);
        } else {
            f[static_cast<long long>(i) * k.N + c] = w * r * (1.0 + h);
        }
    });
}

// Copy float64 f[Q][N] into storage, and back.
template <class M, class P>
__global__ __launch_bounds__(kBlock) void k_set_pop(const double* __restrict__ fin,
                                                    typename P::S* __restrict__ f, KParams k) {
    const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= k.N) return;
    static_for<M::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int g = M::table.group[i];
        const double val = fin[static_cast<long long>(i) * k.N + c];
        if constexpr (P::shifted)
            f[static_cast<long long>(i) * k.N + c] = static_cast<float>(val - k.W[g] * k.rho0);
        else
            f[static_cast<long long>(i) * k.N + c] = val;
    });
}

template <class M, class P>
__global__ __launch_bounds__(kBlock) void k_get_pop(const typename P::S* __restrict__ f,
                                                    double* __restrict__ fout, KParams k) {
    const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= k.N) return;
    static_for<M::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int g = M::table.group[i];
        const double val = static_cast<double>(f[static_cast<long long>(i) * k.N + c]);
        fout[static_cast<long long>(i) * k.N + c] = P::shifted ? val + k.W[g] * k.rho0 : val;
    });
}

// Raw float64 sums of one cell: sum v, sum v e, sum v |e|^2 of the stored values.
template <class M, class S>
__device__ __forceinline__ void cell_sums(const S* __restrict__ f, const KParams& k, long long c,
                                          double& m0, double (&j)[3], double& en) {
    m0 = 0.0;
    j[0] = j[1] = j[2] = 0.0;
    en = 0.0;
    static_for<M::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = M::table.e[i][0], ey = M::table.e[i][1], ez = M::table.e[i][2];
        constexpr int ee = M::table.e2[M::table.group[i]];
        const double val = static_cast<double>(f[static_cast<long long>(i) * k.N + c]);
        m0 += val;
        if constexpr (ex != 0) j[0] += double(ex) * val;
        if constexpr (ey != 0) j[1] += double(ey) * val;
        if constexpr (ez != 0) j[2] += double(ez) * val;
        if constexpr (ee != 0) en += double(ee) * val;
    });
}

template <class M, class P>
__global__ __launch_bounds__(kBlock) void k_moments(const typename P::S* __restrict__ f,
                                                    double* __restrict__ rho, double* __restrict__ U,
                                                    double* __restrict__ T, KParams k) {
    constexpr int D = M::D;
    const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= k.N) return;
    double m0, j[3], en;
    cell_sums<M>(f, k, c, m0, j, en);
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
template <class M, class P>
__global__ __launch_bounds__(kBlock) void k_conservation(const typename P::S* __restrict__ f,
                                                         KParams k, double* __restrict__ partials) {
    constexpr int D = M::D;
    double acc[D + 2];
    static_for<D + 2>([&](auto QI) { acc[decltype(QI)::value] = 0.0; });
    const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < k.N;
         c += stride) {
        double m0, j[3], en;
        cell_sums<M>(f, k, c, m0, j, en);
        acc[0] += m0;
        for (int a = 0; a < D; ++a) acc[1 + a] += j[a];
        acc[D + 1] += 0.5 * en;
    }
    block_sum<D + 2>(acc, partials + static_cast<long long>(blockIdx.x) * (D + 2), false);
}

__global__ __launch_bounds__(kBlock) void k_fill_zero(double* p, long long n) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// out[q] = sum_j part[j*stride + q] for q < count, one block, fixed order.
__global__ __launch_bounds__(kBlock) void k_sum_partials(const double* __restrict__ part,
                                                         long long n, int stride, int count,
                                                         double* __restrict__ out) {
    __shared__ double sh[kBlock];
    for (int q = 0; q < count; ++q) {
        double s = 0.0;
        for (long long j = threadIdx.x; j < n; j += blockDim.x) s += part[j * stride + q];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if (static_cast<int>(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[q] = sh[0];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Adjoint.
//
// lambda^n_i(x) = dL/drho_n(x) for every i; partK[block] = sum dL/drho_n * rho_n.
template <class M, class P>
__global__ __launch_bounds__(kBlock) void k_lambda_init(const typename P::S* __restrict__ fn,
                                                        const double* __restrict__ dLdrho,
                                                        typename P::S* __restrict__ lam,
                                                        KParams k, double* __restrict__ partK) {
    using S = typename P::S;
    const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    double acc[1] = {0.0};
    if (c < k.N) {
        const double g = dLdrho[c];
        double m0 = 0.0;
        static_for<M::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            m0 += static_cast<double>(fn[static_cast<long long>(i) * k.N + c]);
            lam[static_cast<long long>(i) * k.N + c] = static_cast<S>(g);
        });
        const double r = P::shifted ? k.rho0 + m0 : m0;
        acc[0] = g * r;
    }
    block_sum<1>(acc, partK + blockIdx.x, false);
}

// Derivative coefficients of P = 1 + h with respect to s, u2 and d:
//   P_s  = a1 + s (2 a2 + s (1/2 + s/6))
//   P_u2 = b0 + s (-1/2 - s/4),          b0 = -1/2 + u2/4 + d (D + 2 - X)/4
//   P_d  = c0 + s (c1 + s c2),            c0 = (X - D)/2 + (D + 2 - X) u2/4
//                                              + d (X^2 - 2 (D + 2) X + D (D + 2))/4
//                                         c1 = (X - D - 2)/2, c2 = (X - D - 4)/4
template <int D, class R>
struct HermD {
    R a0, a1, a2, b0, c0, c1, c2;
    __device__ __forceinline__ void set(R X, R u2, R d) {
        const R Dr = R(D);
        a0 = R(0.5) * (d * (X - Dr) - u2) +
             R(1.0 / 24.0) * (R(3) * u2 * u2 + R(6) * d * (Dr + R(2) - X) * u2 +
                              R(3) * d * d * (X * X - R(2) * (Dr + R(2)) * X + Dr * (Dr + R(2))));
        a1 = R(1) - R(0.5) * u2 + R(0.5) * d * (X - Dr - R(2));
        a2 = R(0.5) - R(0.25) * u2 + R(0.25) * d * (X - Dr - R(4));
        b0 = R(-0.5) + R(0.25) * u2 + R(0.25) * d * (Dr + R(2) - X);
        c1 = R(0.5) * (X - Dr - R(2));
        c2 = R(0.25) * (X - Dr - R(4));
        c0 = R(0.5) * (X - Dr) + R(0.25) * (Dr + R(2) - X) * u2 +
             R(0.25) * d * (X * X - R(2) * (Dr + R(2)) * X + Dr * (Dr + R(2)));
    }
};

// One transposed step.  mu_i = lambda^{t+1}_i(x + e_i); the moments of f^t at x
// come from the recomputation.  partA[block] += sum_x rho sum_i mu_i w_i P_i.
template <class M, class P>
__global__ __launch_bounds__(kBlock) void k_adjoint(const typename P::S* __restrict__ lsrc,
                                                    typename P::S* __restrict__ ldst,
                                                    const typename P::S* __restrict__ mom,
                                                    KParams k, double* __restrict__ partA) {
    using S = typename P::S;
    using R = S;
    constexpr int Q = M::Q;
    constexpr int G = M::G;
    constexpr int D = M::D;
    const Cell cl = row_cell(k);

    S mu[Q];
    gather<M, -1>(lsrc, k, cl, mu);

    const R m0 = mom[cl.c];
    const R ux = mom[k.N + cl.c];
    const R uy = mom[2 * k.N + cl.c];
    const R uz = (D == 3) ? mom[3 * k.N + cl.c] : R(0);
    const R d = mom[(D + 1) * k.N + cl.c];
    const R rho = P::shifted ? kp_rho0<R>(k) + m0 : m0;
    const R T0 = kp_T0<R>(k);
    const R invT0 = kp_invT0<R>(k);
    const R omega = kp_omega<R>(k);
    const R omc = R(1) - omega;
    const R usq = ux * ux + uy * uy + uz * uz;
    const R utx = ux * invT0, uty = uy * invT0, utz = uz * invT0;
    const R u2 = usq * invT0;

    HermD<D, R> hc[G];
    static_for<G>([&](auto GI) {
        constexpr int g = decltype(GI)::value;
        hc[g].set(kp_x<R>(k, g), u2, d);
    });

    R s0 = R(0), su2 = R(0), sd = R(0), ssx = R(0), ssy = R(0), ssz = R(0);
    static_for<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int g = M::table.group[i];
        constexpr int ex = M::table.e[i][0], ey = M::table.e[i][1], ez = M::table.e[i][2];
        const HermD<D, R>& c = hc[g];
        const R s = edot<ex, ey, ez>(utx, uty, utz);
        const R mw = mu[i] * kp_w<R>(k, g);
        const R p = R(1) + c.a0 + s * (c.a1 + s * (c.a2 + s * (R(1.0 / 6.0) + s * R(1.0 / 24.0))));
        const R ps = c.a1 + s * (R(2) * c.a2 + s * (R(0.5) + s * R(1.0 / 6.0)));
        const R pu = c.b0 + s * (R(-0.5) - s * R(0.25));
        const R pd = c.c0 + s * (c.c1 + s * c.c2);
        s0 = fma(mw, p, s0);
        su2 = fma(mw, pu, su2);
        sd = fma(mw, pd, sd);
        const R t = mw * ps;
        if constexpr (ex != 0) ssx = fma(R(ex), t, ssx);
        if constexpr (ey != 0) ssy = fma(R(ey), t, ssy);
        if constexpr (ez != 0) ssz = fma(R(ez), t, ssz);
    });

    // Chain rule from (rho, U, T) to (rho, j = rho U, E = sum f |e|^2).
    const R rT = rho * invT0;
    const R aux = rT * (ssx + R(2) * ux * su2);
    const R auy = rT * (ssy + R(2) * uy * su2);
    const R auz = rT * (ssz + R(2) * uz * su2);
    const R at = rT * sd;
    const R invr = R(1) / rho;
    const R Tm = T0 * (R(1) + d);
    const R grho = s0 - invr * (aux * ux + auy * uy + auz * uz) +
                   at * (usq - R(D) * Tm) * invr * R(1.0 / D);
    const R k2 = R(2.0 / D) * at * invr;
    const R gjx = omega * (aux * invr - k2 * ux);
    const R gjy = omega * (auy * invr - k2 * uy);
    const R gjz = omega * (auz * invr - k2 * uz);
    const R ge = omega * at * invr * R(1.0 / D);
    const R gr = omega * grho;

    static_for<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ex = M::table.e[i][0], ey = M::table.e[i][1], ez = M::table.e[i][2];
        constexpr int ee = M::table.e2[M::table.group[i]];
        R hv = gr;
        if constexpr (ee != 0) hv = fma(R(ee), ge, hv);
        if constexpr (ex != 0) hv = fma(R(ex), gjx, hv);
        if constexpr (ey != 0) hv = fma(R(ey), gjy, hv);
        if constexpr (ez != 0) hv = fma(R(ez), gjz, hv);
        if (cl.active) ldst[static_cast<long long>(i) * k.N + cl.c] = fma(omc, mu[i], hv);
    });

    double acc[1] = {cl.active ? static_cast<double>(rho) * static_cast<double>(s0) : 0.0};
    block_sum<1>(acc, partA + blockIdx.x, true);
}

// dL/dT_init(x) = sum_i lambda^0_i(x) d f_i^eq / dT at the initial fields.
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
    const double invT0 = 1.0 / k.T0;
    const double d = T[c] * invT0 - 1.0;
    const double u2 = (ux * ux + uy * uy + uz * uz) * invT0;
    const double utx = ux * invT0, uty = uy * invT0, utz = uz * invT0;
    HermD<D, double> hc[G];
    static_for<G>([&](auto GI) {
        constexpr int g = decltype(GI)::value;
        hc[g].set(k.X[g], u2, d);
    });
    double sd = 0.0;
    static_for<M::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int g = M::table.group[i];
        constexpr int ex = M::table.e[i][0], ey = M::table.e[i][1], ez = M::table.e[i][2];
        const double s = edot<ex, ey, ez>(utx, uty, utz);
        const double pd = hc[g].c0 + s * (hc[g].c1 + s * hc[g].c2);
        sd += static_cast<double>(lam[static_cast<long long>(i) * k.N + c]) * k.W[g] * pd;
    });
    dT[c] = r * invT0 * sd;
}

template <class F>
hipError_t with_types(ModelId m, Prec p, F&& f) {
    if (m == ModelId::D2Q33) {
        if (p == Prec::F64) return f(D2Q33{}, F64T{});
        return f(D2Q33{}, F32ST{});
    }
    if (p == Prec::F64) return f(D3Q95{}, F64T{});
    return f(D3Q95{}, F32ST{});
}

inline unsigned cell_blocks(long long N) {
    return static_cast<unsigned>((N + kBlock - 1) / kBlock);
}

}  // namespace

RowLaunch row_launch(int nx, long long rows, int max_threads) {
    RowLaunch r;
    const int maxb = max_threads < kBlock ? max_threads : kBlock;
    r.chunks = (nx + maxb - 1) / maxb;
    const int per = (nx + r.chunks - 1) / r.chunks;
    r.bx = ((per + 63) / 64) * 64;
    r.blocks = rows * r.chunks;
    return r;
}

int reduce_blocks(long long N) {
    long long b = (N + kBlock - 1) / kBlock;
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return static_cast<int>(b);
}

long long step_blocks(ModelId, Prec, const KParams& kp) {
    return static_cast<long long>(kp.ny) * kp.nz * kp.chunks;
}

hipError_t launch_init(ModelId m, Prec p, const KParams& kp, const double* rho, const double* U,
                       const double* T, void* f, hipStream_t s) {
    return with_types(m, p, [&](auto M_, auto P_) {
        using M = decltype(M_);
        using P = decltype(P_);
        hipLaunchKernelGGL((k_init<M, P>), dim3(cell_blocks(kp.N)), dim3(kBlock), 0, s, rho, U, T,
                           static_cast<typename P::S*>(f), kp);
        return hipGetLastError();
    });
}

hipError_t launch_set_pop(ModelId m, Prec p, const KParams& kp, const double* fin, void* f,
                          hipStream_t s) {
    return with_types(m, p, [&](auto M_, auto P_) {
        using M = decltype(M_);
        using P = decltype(P_);
        hipLaunchKernelGGL((k_set_pop<M, P>), dim3(cell_blocks(kp.N)), dim3(kBlock), 0, s, fin,
                           static_cast<typename P::S*>(f), kp);
        return hipGetLastError();
    });
}

hipError_t launch_get_pop(ModelId m, Prec p, const KParams& kp, const void* f, double* fout,
                          hipStream_t s) {
    return with_types(m, p, [&](auto M_, auto P_) {
        using M = decltype(M_);
        using P = decltype(P_);
        hipLaunchKernelGGL((k_get_pop<M, P>), dim3(cell_blocks(kp.N)), dim3(kBlock), 0, s,
                           static_cast<const typename P::S*>(f), fout, kp);
        return hipGetLastError();
    });
}

hipError_t launch_step(ModelId m, Prec p, const KParams& kp, const void* src, void* dst,
                       void* mom_out, hipStream_t s) {
    const long long blocks = step_blocks(m, p, kp);
    return with_types(m, p, [&](auto M_, auto P_) {
        using M = decltype(M_);
        using P = decltype(P_);
        using S = typename P::S;
        if (mom_out) {
            hipLaunchKernelGGL((k_step<M, P, true>), dim3(static_cast<unsigned>(blocks)),
                               dim3(kp.bx), 0, s, static_cast<const S*>(src), static_cast<S*>(dst),
                               kp, static_cast<S*>(mom_out));
        } else {
            hipLaunchKernelGGL((k_step<M, P, false>), dim3(static_cast<unsigned>(blocks)),
                               dim3(kp.bx), 0, s, static_cast<const S*>(src), static_cast<S*>(dst),
                               kp, static_cast<S*>(nullptr));
        }
        return hipGetLastError();
    });
}

hipError_t launch_moments(ModelId m, Prec p, const KParams& kp, const void* f, double* rho,
                          double* U, double* T, hipStream_t s) {
    return with_types(m, p, [&](auto M_, auto P_) {
        using M = decltype(M_);
        using P = decltype(P_);
        hipLaunchKernelGGL((k_moments<M, P>), dim3(cell_blocks(kp.N)), dim3(kBlock), 0, s,
                           static_cast<const typename P::S*>(f), rho, U, T, kp);
        return hipGetLastError();
    });
}

hipError_t launch_conservation(ModelId m, Prec p, const KParams& kp, const void* f,
                               double* partials, double* out, hipStream_t s) {
    const int nb = reduce_blocks(kp.N);
    const int D = (m == ModelId::D2Q33) ? 2 : 3;
    hipError_t e = with_types(m, p, [&](auto M_, auto P_) {
        using M = decltype(M_);
        using P = decltype(P_);
        hipLaunchKernelGGL((k_conservation<M, P>), dim3(nb), dim3(kBlock), 0, s,
                           static_cast<const typename P::S*>(f), kp, partials);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    return launch_sum_partials(partials, nb, D + 2, D + 2, out, s);
}

hipError_t launch_fill_zero(double* p, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_zero, dim3(cell_blocks(n)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double* part, long long n, int stride, int count,
                               double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, part, n, stride, count, out);
    return hipGetLastError();
}

hipError_t launch_lambda_init(ModelId m, Prec p, const KParams& kp, const void* fn,
                              const double* dLdrho, void* lam, double* partK, hipStream_t s) {
    return with_types(m, p, [&](auto M_, auto P_) {
        using M = decltype(M_);
        using P = decltype(P_);
        using S = typename P::S;
        hipLaunchKernelGGL((k_lambda_init<M, P>), dim3(cell_blocks(kp.N)), dim3(kBlock), 0, s,
                           static_cast<const S*>(fn), dLdrho, static_cast<S*>(lam), kp, partK);
        return hipGetLastError();
    });
}

hipError_t launch_adjoint_step(ModelId m, Prec p, const KParams& kp, const void* lam_src,
                               void* lam_dst, const void* mom, double* partA, hipStream_t s) {
    const long long blocks = step_blocks(m, p, kp);
    return with_types(m, p, [&](auto M_, auto P_) {
        using M = decltype(M_);
        using P = decltype(P_);
        using S = typename P::S;
        hipLaunchKernelGGL((k_adjoint<M, P>), dim3(static_cast<unsigned>(blocks)), dim3(kp.bx), 0,
                           s, static_cast<const S*>(lam_src), static_cast<S*>(lam_dst),
                           static_cast<const S*>(mom), kp, partA);
        return hipGetLastError();
    });
}

hipError_t launch_dT_init(ModelId m, Prec p, const KParams& kp, const void* lam0,
                          const double* rho, const double* U, const double* T, double* dT,
                          hipStream_t s) {
    return with_types(m, p, [&](auto M_, auto P_) {
        using M = decltype(M_);
        using P = decltype(P_);
        hipLaunchKernelGGL((k_dT_init<M, P>), dim3(cell_blocks(kp.N)), dim3(kBlock), 0, s,
                           static_cast<const typename P::S*>(lam0), rho, U, T, dT, kp);
        return hipGetLastError();
    });
}

}  // namespace lbm
